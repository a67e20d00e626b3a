// One time step with contact for one system (Sec. 4.1 "Collision
// resolution"), templated on the scalar (float, double, or their dual
// numbers for exact step Jacobians).  Host and device code: the kernels in
// contact.hip run it per lane; a host build runs the same statements.
#pragma once

#include <cfloat>
#include <cmath>

#include "../../include/abadj.h"
#include "dual.h"

namespace aba_contact {

using aba::Dual;

constexpr int kNL = SIM_CONTACT_MAX_LINKS;
constexpr int kNC = SIM_CONTACT_MAX_SPHERES;
constexpr int kNR = 3 * kNC;
constexpr int kNQ = 7 + (kNL - 1);
constexpr int kNV = 6 + (kNL - 1);
constexpr int kNX = kNQ + kNV;
constexpr int kParLink = 25;  // E_T 9, r_T 3, axis 3, mass 1, com 3, Ic 6
constexpr int kParSphere = 4; // centre 3, radius 1

struct CTopo {
  int n, nq, nv, nu, nc, niter, np;
  int parent[kNL], jtype[kNL], qi[kNL], vi[kNL], ui[kNL];
  int clink[kNC];
  double mu, beta, g[3];
  int has_limits;
  double lim[kNL][4];  // joint limits of the 1-dof joints: lo, hi, stiffness, damping
};

// ---- scalar helpers (plain and dual) --------------------------------------

ABA_HD float val(float x) { return x; }
ABA_HD double val(double x) { return x; }
template <typename R>
ABA_HD R val(const Dual<R>& x) { return x.v; }

ABA_HD void sin_cos(float x, float& s, float& c) { s = sinf(x); c = cosf(x); }
ABA_HD void sin_cos(double x, double& s, double& c) { s = sin(x); c = cos(x); }
template <typename R>
ABA_HD void sin_cos(const Dual<R>& x, Dual<R>& s, Dual<R>& c) {
  R sv, cv;
  sin_cos(x.v, sv, cv);
  s = Dual<R>(sv, cv * x.d);
  c = Dual<R>(cv, -sv * x.d);
}
ABA_HD float sq_root(float x) { return sqrtf(x); }
ABA_HD double sq_root(double x) { return sqrt(x); }
template <typename R>
ABA_HD Dual<R> sq_root(const Dual<R>& x) {
  const R s = sq_root(x.v);
  return Dual<R>(s, x.d / (R(2) * s));
}

// a * b + c as one fused multiply-add.  The sums of products written with
// it round the same way in every kernel variant that runs them: left to the
// compiler, a sum whose first two terms are products (a b + c d, as an
// unrolled sum from zero becomes) may be fused either way round, and which
// way can differ between two builds of the same statements.
ABA_HD float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
ABA_HD double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename T>  // dual numbers, the operation counter
ABA_HD T fmadd(const T& a, const T& b, const T& c) { return a * b + c; }
// A term of a sum unrolled past its true length: live is false past it.
// The kernels compute every term (one past the true length multiplies a zero
// by a finite entry and adds nothing), so no load waits on a condition; the
// operation counter overloads these to count only the live terms.
template <typename T>
ABA_HD T fmadd_pad(const T& a, const T& b, const T& c, bool) { return fmadd(a, b, c); }
template <typename T>
ABA_HD T mul_pad(const T& a, const T& b, bool) { return a * b; }
template <typename T>
ABA_HD T add_pad(const T& a, const T& b, bool) { return a + b; }
template <typename T>
ABA_HD T sub_pad(const T& a, const T& b, bool) { return a - b; }

template <typename R> struct Big;
template <> struct Big<float> { static constexpr float v = FLT_MAX; };
template <> struct Big<double> { static constexpr double v = 1e300; };
template <typename T> struct RealOf { using type = T; };
template <typename R> struct RealOf<Dual<R>> { using type = R; };

// Joint-limit torque of a 1-dof joint: outside [lo, hi] a one-sided spring
// and damper, -k (q - hi) - d qd above, -k (q - lo) - d qd below; zero
// inside.  The side is decided on the value of q against the limits as the
// scalar type holds them.
template <typename S>
ABA_HD S limit_torque(const CTopo& tp, int i, const S& q, const S& qd) {
  const double* L = tp.lim[i];
  if (val(q) > val(S(L[1]))) return -(S(L[2]) * (q - S(L[1]))) - S(L[3]) * qd;
  if (val(q) < val(S(L[0]))) return -(S(L[2]) * (q - S(L[0]))) - S(L[3]) * qd;
  return S(0);
}

// ---- 3-vector and spatial helpers (motion [w; v], force [n; f]) ------------

template <typename S>
ABA_HD void cross3(const S* a, const S* b, S* o) {
  const S x = a[1] * b[2] - a[2] * b[1], y = a[2] * b[0] - a[0] * b[2], z = a[0] * b[1] - a[1] * b[0];
  o[0] = x; o[1] = y; o[2] = z;
}
// y = X x for X = [E 0; -E[r]x E]: y_w = E x_w, y_v = E (x_v - r x x_w)
template <typename S>
ABA_HD void x_motion(const S* E, const S* r, const S* x, S* y) {
  S t[3], o[6];
  cross3(r, x, t);
  for (int a = 0; a < 3; ++a) {
    o[a] = E[3 * a] * x[0] + E[3 * a + 1] * x[1] + E[3 * a + 2] * x[2];
    o[3 + a] = E[3 * a] * (x[3] - t[0]) + E[3 * a + 1] * (x[4] - t[1]) + E[3 * a + 2] * (x[5] - t[2]);
  }
  for (int k = 0; k < 6; ++k) y[k] = o[k];
}
// y = X^T f: y_f = E^T f_f, y_n = E^T f_n + r x y_f
template <typename S>
ABA_HD void xt_force(const S* E, const S* r, const S* f, S* y) {
  S o[6];
  for (int b = 0; b < 3; ++b) {
    o[b] = E[b] * f[0] + E[3 + b] * f[1] + E[6 + b] * f[2];
    o[3 + b] = E[b] * f[3] + E[3 + b] * f[4] + E[6 + b] * f[5];
  }
  S t[3];
  cross3(r, o + 3, t);
  for (int k = 0; k < 3; ++k) y[k] = o[k] + t[k];
  for (int k = 0; k < 3; ++k) y[3 + k] = o[3 + k];
}
template <typename S>
ABA_HD void mat6_vec(const S* M, const S* x, S* y) {
  for (int a = 0; a < 6; ++a) {
    S s = M[6 * a] * x[0];
    for (int b = 1; b < 6; ++b) s = s + M[6 * a + b] * x[b];
    y[a] = s;
  }
}

template <typename R>
struct Par {  // one system's parameters, stored [np][batch]
  const R* P;
  size_t B;
  int s;
  ABA_HD R operator()(int k) const { return P[(size_t)k * B + s]; }
};

template <typename S>
struct Work {
  S E[kNL][9], r[kNL][3];    // parent -> link transform
  S Ew[kNL][9], ow[kNL][3];  // world -> link rotation, link origin in world coordinates
  S ax[kNL][3];              // unit joint axis
  S v[kNL][6], c[kNL][6], pA[kNL][6], IA[kNL][36], U[kNL][6], Dinv[kNL], u[kNL], a[kNL][6];
  S L0[36], D0[6];           // LDL^T of the free root's articulated inertia
  S J[kNR][kNV], MJ[kNV][kNR];
  S A[kNR * kNR], b[kNR], x[kNR];
  // pads the struct to an odd number of scalars, so that lanes holding
  // consecutive Work records in LDS fall on distinct banks
  S pad_;
};

// What the step's adjoint needs beyond Work: the accelerations, the
// contact set and the two solves' sweep vectors (filled when contact_step
// gets a record).
constexpr int kSweepMax = 64;  // PGS sweeps a recorded step may run
template <typename S>
struct Rec {
  S qdd[kNV];               // accelerations (a free root's: true body-frame)
  S qdm[kNV];               // qd_minus = qd + dt qdd
  int na, r, nk, nkn;       // active contacts, rows, kept rows, kept normal rows
  int act[kNC], keep[kNR], kn[kNC];
  S phi[kNC], cl[kNC][3], pw[kNC][3];
  S lamn[kNC];              // normal impulses of the first solve, per active contact
  S x1[kSweepMax + 1][kNC]; // first solve: x at the start of every sweep (and the result)
  S x2[kSweepMax + 1][kNR]; // second solve
};

// The articulated quantities that the unit-impulse responses (M^-1 J^T)
// and the adjoint's solves with M read, with the responses' scratch: a
// per-lane copy that the gradient kernel keeps in LDS, where those long
// sweeps see LDS rather than private-memory latency.  An odd number of
// scalars, so that consecutive lanes' copies fall on distinct banks.
template <typename S>
struct Art {
  S E[kNL][9], r[kNL][3], ax[kNL][3], U[kNL][6], Dinv[kNL], L0[36], D0[6];
  S Ib[kNL][10];  // mass, centre of mass (3), inertia about it (xx yy zz xy xz yz)
  S pA[kNL][6], a[kNL][6], u[kNL], s3[kNL][6];  // scratch of the responses and of the adjoint's solves
  S pad_;
};

// unit quaternion (x, y, z, w) -> rotation matrix (body -> world), row-major
template <typename S>
ABA_HD void quat_R(const S* qt, S* R) {
  const S x = qt[0], y = qt[1], z = qt[2], w = qt[3];
  const S d = w * w - (x * x + y * y + z * z);
  const S v[3] = {x, y, z};
  const S two = S(2);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[3 * i + j] = two * v[i] * v[j];
  for (int i = 0; i < 3; ++i) R[4 * i] = R[4 * i] + d;
  R[1] = R[1] - two * w * z; R[2] = R[2] + two * w * y;
  R[3] = R[3] + two * w * z; R[5] = R[5] - two * w * x;
  R[6] = R[6] - two * w * y; R[7] = R[7] + two * w * x;
}

// LDL^T of a symmetric positive definite 6x6 (unit lower L below the diagonal)
template <typename S>
ABA_HD void ldl6(const S* M, S* L, S* D) {
  for (int k = 0; k < 36; ++k) L[k] = M[k];
  for (int j = 0; j < 6; ++j) {
    S d = L[7 * j];
    for (int k = 0; k < j; ++k) d = d - L[6 * j + k] * L[6 * j + k] * D[k];
    D[j] = d;
    for (int i = j + 1; i < 6; ++i) {
      S s = L[6 * i + j];
      for (int k = 0; k < j; ++k) s = s - L[6 * i + k] * L[6 * j + k] * D[k];
      L[6 * i + j] = s / d;
    }
  }
}
template <typename S>
ABA_HD void ldl6_solve(const S* L, const S* D, const S* rhs, S* x) {
  S y[6];
  for (int i = 0; i < 6; ++i) {
    S s = rhs[i];
    for (int k = 0; k < i; ++k) s = s - L[6 * i + k] * y[k];
    y[i] = s;
  }
  for (int i = 5; i >= 0; --i) {
    S s = y[i] / D[i];
    for (int k = i + 1; k < 6; ++k) s = s - L[6 * k + i] * x[k];
    x[i] = s;
  }
}

// projected Gauss-Seidel on the rows idx[0..m) of A (leading dimension r);
// sweeps (nullable, stride ld): x at the start of every sweep and the result
template <typename S>
ABA_HD void pgs(int m, const int* idx, int r, const S* A, const S* b, const S* lo, const S* hi, int niter, S* x,
                S* sweeps = nullptr, int ld = 0) {
  // x in registers, rows and columns unrolled over kNR: the kept rows'
  // indices, 0 beyond m, address valid entries of A, and x stays zero beyond
  // m, so every term of a row's sum runs with no condition (past m it adds
  // zero, the same sum in the same order) and the row's loads issue together
  int ix[kNR];
#pragma unroll
  for (int i = 0; i < kNR; ++i) ix[i] = i < m ? idx[i] : 0;
  S xr[kNR];
#pragma unroll
  for (int i = 0; i < kNR; ++i) xr[i] = S(0);
  for (int it = 0; it < niter; ++it) {
    if (sweeps) {
#pragma unroll
      for (int i = 0; i < kNR; ++i)
        if (i < m) sweeps[it * ld + i] = xr[i];
    }
#pragma unroll
    for (int i = 0; i < kNR; ++i) {
      if (i >= m) continue;
      const S* Ai = A + ix[i] * r;
      S d = S(0);
#pragma unroll
      for (int j = 0; j < kNR; ++j)
        if (j != i) d = fmadd_pad(Ai[ix[j]], xr[j], d, j < m);
      S y = -(b[ix[i]] + d) / Ai[ix[i]];
      if (val(y) < val(lo[i])) y = lo[i];
      else if (val(y) > val(hi[i])) y = hi[i];
      xr[i] = y;
    }
  }
#pragma unroll
  for (int i = 0; i < kNR; ++i)
    if (i < m) x[i] = xr[i];
  if (sweeps)
    for (int i = 0; i < m; ++i) sweeps[niter * ld + i] = x[i];
}

// A compact working copy of one Gauss-Seidel problem, element k at p[k * st]
// (the kernels give every lane its own column of an LDS block, the host a
// plain array): the kept rows' block of A (m x m), b, the bounds, x, the two
// sweep vectors the reverse reads, and the reverse's adjoints of A, b and
// the bounds (that of x stays in registers).  Every access
// of the sweeps then reads this copy directly instead of going through the
// kept-row index into the full record.
template <typename S>
struct PgsStage {
  S* p;
  int st;
  ABA_HD S& operator[](int k) const { return p[(size_t)k * st]; }
};
constexpr int kStA = 0, kStB = kNR * kNR, kStLo = kStB + kNR, kStHi = kStLo + kNR, kStX = kStHi + kNR,
              kStXe = kStX + kNR, kStAb = kStXe + kNR, kStBb = kStAb + kNR * kNR, kStLob = kStBb + kNR,
              kStHib = kStLob + kNR, kStage = kStHib + kNR;

// pgs on a staged copy: the same statements in the same order, so the
// result is bitwise that of pgs.
template <typename S>
ABA_HD void pgs_staged(int m, const int* idx, int r, const S* A, const S* b, const S* lo, const S* hi, int niter,
                       S* x, S* sweeps, int ld, const PgsStage<S>& g) {
  // rows of the block at stride kNR, zero beyond m; x in registers (zero
  // beyond m), rows unrolled over kNR and predicated on m, every row's sum
  // over all kNR columns with no condition (the terms beyond m add zero), so
  // that a row's loads issue together
  // (the kept rows' indices, 0 beyond m, address a valid entry of A, so the
  // copy reads A with no condition and its loads issue together)
  int ix[kNR];
#pragma unroll
  for (int i = 0; i < kNR; ++i) ix[i] = i < m ? idx[i] : 0;
#pragma unroll
  for (int i = 0; i < kNR; ++i)
#pragma unroll
    for (int j = 0; j < kNR; ++j) {
      const S aij = A[ix[i] * r + ix[j]];
      g[kStA + i * kNR + j] = (i < m && j < m) ? aij : S(0);
    }
  for (int i = 0; i < m; ++i) {
    g[kStB + i] = b[idx[i]];
    g[kStLo + i] = lo[i];
    g[kStHi + i] = hi[i];
  }
  S xr[kNR];
#pragma unroll
  for (int i = 0; i < kNR; ++i) xr[i] = S(0);
  for (int it = 0; it < niter; ++it) {
    if (sweeps) {
#pragma unroll
      for (int i = 0; i < kNR; ++i)
        if (i < m) sweeps[it * ld + i] = xr[i];
    }
#pragma unroll
    for (int i = 0; i < kNR; ++i) {
      if (i >= m) continue;
      S d = S(0);
#pragma unroll
      for (int j = 0; j < kNR; ++j)
        if (j != i) d = fmadd_pad(g[kStA + i * kNR + j], xr[j], d, j < m);  // zero beyond m
      S y = -(g[kStB + i] + d) / g[kStA + i * kNR + i];
      if (val(y) < val(g[kStLo + i])) y = g[kStLo + i];
      else if (val(y) > val(g[kStHi + i])) y = g[kStHi + i];
      xr[i] = y;
    }
  }
#pragma unroll
  for (int i = 0; i < kNR; ++i)
    if (i < m) x[i] = xr[i];
  if (sweeps)
    for (int i = 0; i < m; ++i) sweeps[niter * ld + i] = x[i];
}

// M^-1 J^T: the response of the step's articulated system (zero velocity,
// no gravity) to a unit world force along each contact row's direction at
// the contact point, one column of w.MJ per row.  v holds the articulated
// quantities and the scratch (the Work itself, or an Art copy of it).
template <typename S, typename V>
ABA_HD void unit_responses(const CTopo& tp, Work<S>& w, V& v, int na, const int* act, const S (*cl)[3]) {
  const int n = tp.n;
  const int dirs[3] = {1, 0, 2};
  for (int c = 0; c < na; ++c) {
    const int l = tp.clink[act[c]];
    for (int dd = 0; dd < 3; ++dd) {
      for (int i = 0; i < n; ++i)
        for (int k = 0; k < 6; ++k) v.pA[i][k] = S(0);
      S f[3];
      for (int b = 0; b < 3; ++b) f[b] = w.Ew[l][3 * b + dirs[dd]];
      S nmt[3];
      cross3(cl[c], f, nmt);
      for (int k = 0; k < 3; ++k) { v.pA[l][k] = -nmt[k]; v.pA[l][3 + k] = -f[k]; }
      for (int i = n - 1; i >= 0; --i) {
        if (tp.jtype[i] == SIM_JOINT_FREE) continue;
        const int off = tp.jtype[i] == SIM_JOINT_PRISMATIC ? 3 : 0, p = tp.parent[i];
        v.u[i] = -(v.pA[i][off] * v.ax[i][0] + v.pA[i][off + 1] * v.ax[i][1] + v.pA[i][off + 2] * v.ax[i][2]);
        if (p >= 0) {
          const S y = v.Dinv[i] * v.u[i];
          S pa[6], fp[6];
          for (int k = 0; k < 6; ++k) pa[k] = v.pA[i][k] + v.U[i][k] * y;
          xt_force(v.E[i], v.r[i], pa, fp);
          for (int k = 0; k < 6; ++k) v.pA[p][k] = v.pA[p][k] + fp[k];
        }
      }
      for (int i = 0; i < n; ++i) {
        if (tp.jtype[i] == SIM_JOINT_FREE) {
          S rhs[6];
          for (int k = 0; k < 6; ++k) rhs[k] = -v.pA[i][k];
          ldl6_solve(v.L0, v.D0, rhs, v.a[i]);
          for (int k = 0; k < 6; ++k) w.MJ[tp.vi[i] + k][3 * c + dd] = v.a[i][k];
        } else {
          const int p = tp.parent[i], off = tp.jtype[i] == SIM_JOINT_PRISMATIC ? 3 : 0;
          S ap[6];
          if (p < 0) {
            for (int k = 0; k < 6; ++k) ap[k] = S(0);
          } else {
            x_motion(v.E[i], v.r[i], v.a[p], ap);
          }
          S Uap = S(0);
          for (int k = 0; k < 6; ++k) Uap = Uap + v.U[i][k] * ap[k];
          const S qdd = v.Dinv[i] * (v.u[i] - Uap);
          for (int k = 0; k < 6; ++k) v.a[i][k] = ap[k];
          for (int k = 0; k < 3; ++k) v.a[i][off + k] = v.a[i][off + k] + v.ax[i][k] * qdd;
          w.MJ[tp.vi[i]][3 * c + dd] = qdd;
        }
      }
    }
  }
}

// One step with contact from (q, qd) under control u and friction
// coefficient mu (a dual number for its derivative); returns the number of
// active contacts.  rec (nullable, niter <= kSweepMax) keeps what the
// step's adjoint needs.
template <typename S, typename R>
ABA_HD int contact_step(const CTopo& tp, const Par<R>& P, const S* q, const S* qd, const S* u, R dt_, S mu,
                            S* q1, S* qd1, Work<S>& w, Rec<S>* rec = nullptr, PgsStage<S> stage = {nullptr, 0},
                            Art<S>* art = nullptr) {
  using Rl = typename RealOf<S>::type;
  const int n = tp.n, nv = tp.nv;
  const S dt = S(dt_);
  // ---- pass 1: poses, velocities, bias forces
  for (int i = 0; i < n; ++i) {
    const int p = tp.parent[i], pb = kParLink * i;
    S vJ[6];
    if (tp.jtype[i] == SIM_JOINT_FREE) {
      S Rm[9];
      quat_R(q + tp.qi[i] + 3, Rm);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) w.E[i][3 * a + b] = Rm[3 * b + a];
      for (int k = 0; k < 3; ++k) w.r[i][k] = q[tp.qi[i] + k];
      for (int k = 0; k < 6; ++k) { w.v[i][k] = qd[tp.vi[i] + k]; w.c[i][k] = S(0); }
    } else {
      S a[3];
      const R an = R(1) / sq_root(P(pb + 12) * P(pb + 12) + P(pb + 13) * P(pb + 13) + P(pb + 14) * P(pb + 14));
      for (int k = 0; k < 3; ++k) { a[k] = S(P(pb + 12 + k) * an); w.ax[i][k] = a[k]; }
      const S qj = q[tp.qi[i]], qdj = qd[tp.vi[i]];
      S ET[9];
      for (int k = 0; k < 9; ++k) ET[k] = S(P(pb + k));
      for (int k = 0; k < 3; ++k) w.r[i][k] = S(P(pb + 9 + k));
      if (tp.jtype[i] == SIM_JOINT_PRISMATIC) {
        for (int k = 0; k < 9; ++k) w.E[i][k] = ET[k];
        for (int b = 0; b < 3; ++b)
          w.r[i][b] = w.r[i][b] + (ET[b] * a[0] + ET[3 + b] * a[1] + ET[6 + b] * a[2]) * qj;
        for (int k = 0; k < 3; ++k) { vJ[k] = S(0); vJ[3 + k] = a[k] * qdj; }
      } else {
        // E_J = I - sin q [a]x + (1 - cos q) [a]x^2
        S sq, cq;
        sin_cos(qj, sq, cq);
        const S omc = S(1) - cq;
        const S K[9] = {S(0), -a[2], a[1], a[2], S(0), -a[0], -a[1], a[0], S(0)};
        S EJ[9];
        for (int r_ = 0; r_ < 3; ++r_)
          for (int c_ = 0; c_ < 3; ++c_) {
            S k2 = K[3 * r_] * K[c_] + K[3 * r_ + 1] * K[3 + c_] + K[3 * r_ + 2] * K[6 + c_];
            EJ[3 * r_ + c_] = (r_ == c_ ? S(1) : S(0)) - sq * K[3 * r_ + c_] + omc * k2;
          }
        for (int r_ = 0; r_ < 3; ++r_)
          for (int c_ = 0; c_ < 3; ++c_)
            w.E[i][3 * r_ + c_] = EJ[3 * r_] * ET[c_] + EJ[3 * r_ + 1] * ET[3 + c_] + EJ[3 * r_ + 2] * ET[6 + c_];
        for (int k = 0; k < 3; ++k) { vJ[k] = a[k] * qdj; vJ[3 + k] = S(0); }
      }
      if (p < 0) {
        for (int k = 0; k < 6; ++k) w.v[i][k] = vJ[k];
      } else {
        x_motion(w.E[i], w.r[i], w.v[p], w.v[i]);
        for (int k = 0; k < 6; ++k) w.v[i][k] = w.v[i][k] + vJ[k];
      }
      // c = v x vJ (motion cross product)
      const S* vv = w.v[i];
      S t1[3], t2[3], t3[3];
      cross3(vv, vJ, t1);
      cross3(vv + 3, vJ, t2);
      cross3(vv, vJ + 3, t3);
      for (int k = 0; k < 3; ++k) { w.c[i][k] = t1[k]; w.c[i][3 + k] = t2[k] + t3[k]; }
    }
    if (p < 0) {
      for (int k = 0; k < 9; ++k) w.Ew[i][k] = w.E[i][k];
      for (int k = 0; k < 3; ++k) w.ow[i][k] = w.r[i][k];
    } else {
      for (int r_ = 0; r_ < 3; ++r_)
        for (int c_ = 0; c_ < 3; ++c_)
          w.Ew[i][3 * r_ + c_] = w.E[i][3 * r_] * w.Ew[p][c_] + w.E[i][3 * r_ + 1] * w.Ew[p][3 + c_] +
                                 w.E[i][3 * r_ + 2] * w.Ew[p][6 + c_];
      for (int a = 0; a < 3; ++a)
        w.ow[i][a] = w.ow[p][a] + w.Ew[p][a] * w.r[i][0] + w.Ew[p][3 + a] * w.r[i][1] + w.Ew[p][6 + a] * w.r[i][2];
    }
    // spatial inertia about the link origin
    const S m = S(P(pb + 15));
    const S cm[3] = {S(P(pb + 16)), S(P(pb + 17)), S(P(pb + 18))};
    const S Ic[6] = {S(P(pb + 19)), S(P(pb + 20)), S(P(pb + 21)), S(P(pb + 22)), S(P(pb + 23)), S(P(pb + 24))};
    S* I = w.IA[i];
    const S cc = cm[0] * cm[0] + cm[1] * cm[1] + cm[2] * cm[2];
    const int dix[3] = {0, 1, 2};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) I[6 * a + b] = -m * cm[a] * cm[b];
    for (int a = 0; a < 3; ++a) I[7 * dix[a]] = I[7 * dix[a]] + m * cc + Ic[a];
    I[1] = I[1] + Ic[3]; I[6] = I[6] + Ic[3];
    I[2] = I[2] + Ic[4]; I[12] = I[12] + Ic[4];
    I[8] = I[8] + Ic[5]; I[13] = I[13] + Ic[5];
    // m [c]x (upper right), its transpose (lower left), m I (lower right)
    const S mc[3] = {m * cm[0], m * cm[1], m * cm[2]};
    const S cx[9] = {S(0), -mc[2], mc[1], mc[2], S(0), -mc[0], -mc[1], mc[0], S(0)};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        I[6 * a + 3 + b] = cx[3 * a + b];
        I[6 * (3 + a) + b] = cx[3 * b + a];
        I[6 * (3 + a) + 3 + b] = (a == b) ? m : S(0);
      }
    // p^A = v x* (I v)
    S h[6];
    mat6_vec(I, w.v[i], h);
    const S* vv = w.v[i];
    S t1[3], t2[3], t3[3];
    cross3(vv, h, t1);
    cross3(vv + 3, h + 3, t2);
    cross3(vv, h + 3, t3);
    for (int k = 0; k < 3; ++k) { w.pA[i][k] = t1[k] + t2[k]; w.pA[i][3 + k] = t3[k]; }
  }
  // ---- pass 2: articulated inertias and bias forces
  for (int i = n - 1; i >= 0; --i) {
    if (tp.jtype[i] == SIM_JOINT_FREE) continue;
    const int off = tp.jtype[i] == SIM_JOINT_PRISMATIC ? 3 : 0;
    const S* a = w.ax[i];
    for (int r_ = 0; r_ < 6; ++r_)
      w.U[i][r_] = w.IA[i][6 * r_ + off] * a[0] + w.IA[i][6 * r_ + off + 1] * a[1] + w.IA[i][6 * r_ + off + 2] * a[2];
    const S D = w.U[i][off] * a[0] + w.U[i][off + 1] * a[1] + w.U[i][off + 2] * a[2];
    w.Dinv[i] = S(1) / D;
    S ui = u[tp.ui[i]];
    if (tp.has_limits) ui = ui + limit_torque(tp, i, q[tp.qi[i]], qd[tp.vi[i]]);
    w.u[i] = ui - (w.pA[i][off] * a[0] + w.pA[i][off + 1] * a[1] + w.pA[i][off + 2] * a[2]);
    const int p = tp.parent[i];
    if (p >= 0) {
      S Ia[36];
      for (int r_ = 0; r_ < 6; ++r_)
        for (int c_ = 0; c_ < 6; ++c_) Ia[6 * r_ + c_] = w.IA[i][6 * r_ + c_] - w.U[i][r_] * w.Dinv[i] * w.U[i][c_];
      S pa[6], Iac[6];
      mat6_vec(Ia, w.c[i], Iac);
      const S y = w.Dinv[i] * w.u[i];
      for (int r_ = 0; r_ < 6; ++r_) pa[r_] = w.pA[i][r_] + Iac[r_] + w.U[i][r_] * y;
      S f[6];
      xt_force(w.E[i], w.r[i], pa, f);
      for (int k = 0; k < 6; ++k) w.pA[p][k] = w.pA[p][k] + f[k];
      // IA_parent += X^T Ia X, column by column
      for (int j = 0; j < 6; ++j) {
        S e[6], xe[6], t[6], col[6];
        for (int k = 0; k < 6; ++k) e[k] = (k == j) ? S(1) : S(0);
        x_motion(w.E[i], w.r[i], e, xe);
        mat6_vec(Ia, xe, t);
        xt_force(w.E[i], w.r[i], t, col);
        for (int k = 0; k < 6; ++k) w.IA[p][6 * k + j] = w.IA[p][6 * k + j] + col[k];
      }
    }
  }
  // ---- pass 3: accelerations; qd_minus = qd + dt qdd
  const S a0[6] = {S(0), S(0), S(0), S(-tp.g[0]), S(-tp.g[1]), S(-tp.g[2])};
  for (int i = 0; i < n; ++i) {
    if (tp.jtype[i] == SIM_JOINT_FREE) {
      ldl6(w.IA[i], w.L0, w.D0);
      S rhs[6];
      for (int k = 0; k < 6; ++k) rhs[k] = -w.pA[i][k];
      ldl6_solve(w.L0, w.D0, rhs, w.a[i]);
      // body-frame gravity E g added to the gravity-free solution
      for (int k = 0; k < 6; ++k) {
        S acc = w.a[i][k];
        if (k >= 3) acc = acc + (w.E[i][3 * (k - 3)] * S(tp.g[0]) + w.E[i][3 * (k - 3) + 1] * S(tp.g[1]) +
                                 w.E[i][3 * (k - 3) + 2] * S(tp.g[2]));
        qd1[tp.vi[i] + k] = qd[tp.vi[i] + k] + dt * acc;
        if (rec) rec->qdd[tp.vi[i] + k] = acc;
      }
    } else {
      const int p = tp.parent[i], off = tp.jtype[i] == SIM_JOINT_PRISMATIC ? 3 : 0;
      S ap[6];
      x_motion(w.E[i], w.r[i], p < 0 ? a0 : w.a[p], ap);
      for (int k = 0; k < 6; ++k) ap[k] = ap[k] + w.c[i][k];
      S Uap = S(0);
      for (int k = 0; k < 6; ++k) Uap = Uap + w.U[i][k] * ap[k];
      const S qdd = w.Dinv[i] * (w.u[i] - Uap);
      for (int k = 0; k < 6; ++k) w.a[i][k] = ap[k];
      for (int k = 0; k < 3; ++k) w.a[i][off + k] = w.a[i][off + k] + w.ax[i][k] * qdd;
      qd1[tp.vi[i]] = qd[tp.vi[i]] + dt * qdd;
      if (rec) rec->qdd[tp.vi[i]] = qdd;
    }
  }
  if (rec)
    for (int k = 0; k < nv; ++k) rec->qdm[k] = qd1[k];
  if (art) {
    for (int i = 0; i < n; ++i) {
      for (int k = 0; k < 9; ++k) art->E[i][k] = w.E[i][k];
      for (int k = 0; k < 3; ++k) { art->r[i][k] = w.r[i][k]; art->ax[i][k] = w.ax[i][k]; }
      for (int k = 0; k < 6; ++k) art->U[i][k] = w.U[i][k];
      art->Dinv[i] = w.Dinv[i];
      for (int k = 0; k < 10; ++k) art->Ib[i][k] = S(P(kParLink * i + 15 + k));
    }
    for (int k = 0; k < 36; ++k) art->L0[k] = w.L0[k];
    for (int k = 0; k < 6; ++k) art->D0[k] = w.D0[k];
  }
  // ---- detection and assembly
  int act[kNC], na = 0;
  S phi[kNC], cl[kNC][3], pw[kNC][3];
  for (int k = 0; k < tp.nc; ++k) {
    const int l = tp.clink[k], sb = kParLink * n + kParSphere * k;
    const S cc[3] = {S(P(sb)), S(P(sb + 1)), S(P(sb + 2))};
    const S rad = S(P(sb + 3));
    const S y = w.ow[l][1] + w.Ew[l][1] * cc[0] + w.Ew[l][4] * cc[1] + w.Ew[l][7] * cc[2];
    const S g = y - rad;
    if (val(g) < Rl(0)) {
      act[na] = k;
      phi[na] = g;
      for (int a = 0; a < 3; ++a) cl[na][a] = cc[a] - rad * w.Ew[l][3 * a + 1];
      for (int a = 0; a < 3; ++a)
        pw[na][a] = w.ow[l][a] + w.Ew[l][a] * cl[na][0] + w.Ew[l][3 + a] * cl[na][1] + w.Ew[l][6 + a] * cl[na][2];
      ++na;
    }
  }
  if (rec) {
    rec->na = na;
    rec->r = 3 * na;
    rec->nk = rec->nkn = 0;
    for (int c = 0; c < na; ++c) {
      rec->act[c] = act[c];
      rec->phi[c] = phi[c];
      rec->lamn[c] = S(0);
      for (int a = 0; a < 3; ++a) {
        rec->cl[c][a] = cl[c][a];
        rec->pw[c][a] = pw[c][a];
      }
    }
  }
  if (na > 0) {
    const int r = 3 * na;
    const int dirs[3] = {1, 0, 2};
    for (int i = 0; i < r; ++i)
      for (int k = 0; k < nv; ++k) w.J[i][k] = S(0);
    for (int c = 0; c < na; ++c) {
      for (int j = tp.clink[act[c]]; j >= 0; j = tp.parent[j]) {
        S d[3];
        for (int k = 0; k < 3; ++k) d[k] = pw[c][k] - w.ow[j][k];
        if (tp.jtype[j] == SIM_JOINT_FREE) {
          for (int e = 0; e < 3; ++e) {
            const S Re[3] = {w.Ew[j][3 * e], w.Ew[j][3 * e + 1], w.Ew[j][3 * e + 2]};
            S col[3];
            cross3(Re, d, col);
            for (int dd = 0; dd < 3; ++dd) {
              w.J[3 * c + dd][tp.vi[j] + e] = col[dirs[dd]];
              w.J[3 * c + dd][tp.vi[j] + 3 + e] = Re[dirs[dd]];
            }
          }
        } else {
          S z[3], col[3];
          for (int b = 0; b < 3; ++b) z[b] = w.Ew[j][b] * w.ax[j][0] + w.Ew[j][3 + b] * w.ax[j][1] + w.Ew[j][6 + b] * w.ax[j][2];
          if (tp.jtype[j] == SIM_JOINT_PRISMATIC) {
            for (int k = 0; k < 3; ++k) col[k] = z[k];
          } else {
            cross3(z, d, col);
          }
          for (int dd = 0; dd < 3; ++dd) w.J[3 * c + dd][tp.vi[j]] = col[dirs[dd]];
        }
      }
    }
    // M^-1 J^T: response to a unit world force along each row's direction at
    // the contact point.  MJ is cleared first: the sums below run over all
    // kNR columns and kNV rows, their unused terms multiplied by zero, which
    // needs those entries finite.
#pragma unroll
    for (int k = 0; k < kNV; ++k)
#pragma unroll
      for (int j = 0; j < kNR; ++j) w.MJ[k][j] = S(0);
    if (art) unit_responses(tp, w, *art, na, act, cl);
    else unit_responses(tp, w, w, na, act, cl);
    // A = J M^-1 J^T, b = J qd_minus + (beta/dt) phi (normal rows)
    const S bdt = S(tp.beta) / dt;
    Rl dmax = Rl(0);
    for (int i = 0; i < r; ++i) {
      // row i of J held in registers, zero beyond nv; the sums over k run
      // over all kNV terms with no condition (a term beyond nv is zero times
      // a cleared entry, adding nothing), three columns of MJ per pass (r is
      // a multiple of 3), so that a pass's loads issue together; a load
      // under a lane-dependent condition would wait on its own
      S Ji[kNV];
#pragma unroll
      for (int k = 0; k < kNV; ++k) {
        const S v = w.J[i][k];
        Ji[k] = k < nv ? v : S(0);
      }
      for (int j0 = 0; j0 < r; j0 += 3) {
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
          const int j = j0 + jj;
          S s = S(0);
#pragma unroll
          for (int k = 0; k < kNV; ++k) s = fmadd_pad(Ji[k], w.MJ[k][j], s, k < nv);
          w.A[i * r + j] = s;
        }
      }
      S s = S(0);
#pragma unroll
      for (int k = 0; k < kNV; ++k)  // qd1 may hold only nv entries: past them qd1[0], times zero
        s = fmadd_pad(Ji[k], qd1[k < nv ? k : 0], s, k < nv);
      w.b[i] = (i % 3 == 0) ? s + bdt * phi[i / 3] : s;
      if (val(w.A[i * r + i]) > dmax) dmax = val(w.A[i * r + i]);
    }
    int keep[kNR], nk = 0, kn[kNC], nkn = 0;
    for (int i = 0; i < r; ++i)
      if (val(w.A[i * r + i]) > Rl(1e-12) * dmax) {
        keep[nk++] = i;
        if (i % 3 == 0) kn[nkn++] = i;
      }
    S lo[kNR], hi[kNR], lamn[kNC], xn[kNC];
    for (int i = 0; i < nkn; ++i) { lo[i] = S(0); hi[i] = S(Big<Rl>::v); }
    if (stage.p) pgs_staged(nkn, kn, r, w.A, w.b, lo, hi, tp.niter, xn, rec ? &rec->x1[0][0] : nullptr, kNC, stage);
    else pgs(nkn, kn, r, w.A, w.b, lo, hi, tp.niter, xn, rec ? &rec->x1[0][0] : nullptr, kNC);
    for (int c = 0; c < na; ++c) lamn[c] = S(0);
    for (int i = 0; i < nkn; ++i) lamn[kn[i] / 3] = xn[i];
    for (int i = 0; i < nk; ++i) {
      if (keep[i] % 3 == 0) {
        lo[i] = S(0);
        hi[i] = S(Big<Rl>::v);
      } else {
        lo[i] = -(mu * lamn[keep[i] / 3]);
        hi[i] = mu * lamn[keep[i] / 3];
      }
    }
    S xk[kNR];
    if (stage.p) pgs_staged(nk, keep, r, w.A, w.b, lo, hi, tp.niter, xk, rec ? &rec->x2[0][0] : nullptr, kNR, stage);
    else pgs(nk, keep, r, w.A, w.b, lo, hi, tp.niter, xk, rec ? &rec->x2[0][0] : nullptr, kNR);
    if (rec) {
      rec->nk = nk;
      rec->nkn = nkn;
      for (int i = 0; i < nk; ++i) rec->keep[i] = keep[i];
      for (int i = 0; i < nkn; ++i) rec->kn[i] = kn[i];
      for (int c = 0; c < na; ++c) rec->lamn[c] = lamn[c];
    }
    for (int j = 0; j < r; ++j) w.x[j] = S(0);
    for (int i = 0; i < nk; ++i) w.x[keep[i]] = xk[i];
    S xr[kNR];
#pragma unroll
    for (int j = 0; j < kNR; ++j) {
      const S v = w.x[j];
      xr[j] = j < r ? v : S(0);
    }
    for (int k = 0; k < nv; ++k) {
      S s = S(0);
#pragma unroll
      for (int j = 0; j < kNR; ++j) s = fmadd_pad(w.MJ[k][j], xr[j], s, j < r);
      qd1[k] = qd1[k] + s;
    }
  }
  // ---- positions from the new velocity
  for (int i = 0; i < n; ++i) {
    if (tp.jtype[i] == SIM_JOINT_FREE) {
      const S* qt = q + tp.qi[i] + 3;
      const S* v1 = qd1 + tp.vi[i];
      S Rm[9];
      quat_R(qt, Rm);
      for (int a = 0; a < 3; ++a)
        q1[tp.qi[i] + a] = q[tp.qi[i] + a] + dt * (Rm[3 * a] * v1[3] + Rm[3 * a + 1] * v1[4] + Rm[3 * a + 2] * v1[5]);
      // quat1 = normalize(quat + dt/2 quat (x) (w1, 0))
      S dq[4];
      dq[3] = -(qt[0] * v1[0] + qt[1] * v1[1] + qt[2] * v1[2]);
      S cr[3];
      cross3(qt, v1, cr);
      for (int k = 0; k < 3; ++k) dq[k] = qt[3] * v1[k] + cr[k];
      S qr[4];
      const S h = S(0.5) * dt;
      for (int k = 0; k < 4; ++k) qr[k] = qt[k] + h * dq[k];
      const S nrm = sq_root(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
      for (int k = 0; k < 4; ++k) q1[tp.qi[i] + 3 + k] = qr[k] / nrm;
    } else {
      q1[tp.qi[i]] = q[tp.qi[i]] + dt * qd1[tp.vi[i]];
    }
  }
  return na;
}

}  // namespace aba_contact
