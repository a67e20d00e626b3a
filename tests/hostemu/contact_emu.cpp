// Test-only host run of the GPU contact step (csrc/contact_step.h): the
// same templated statements the kernels run per lane, for one system at a
// time in double, float or dual numbers.  Lets the CPU test suite compare
// the contact path with the oracle without a GPU.  Never loaded by the
// package.
#include <vector>

#include "../../paper_2109_07719_amd/csrc/contact_adjoint.h"

using namespace aba_contact;
using aba::Dual;

namespace {

CTopo topo(int n, const int* parent, const int* jtype, int nc, const int* clink, double mu, double beta, int niter,
           const double* g, const double* limits) {
  CTopo tp{};
  if (limits) {
    tp.has_limits = 1;
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < 4; ++k) tp.lim[i][k] = limits[4 * i + k];
  }
  tp.n = n;
  tp.nc = nc;
  tp.mu = mu;
  tp.beta = beta;
  tp.niter = niter;
  for (int k = 0; k < 3; ++k) tp.g[k] = g[k];
  int nq = 0, nv = 0, nu = 0;
  for (int i = 0; i < n; ++i) {
    tp.parent[i] = parent[i];
    tp.jtype[i] = jtype[i];
    tp.qi[i] = nq;
    tp.vi[i] = nv;
    tp.ui[i] = nu;
    if (jtype[i] == SIM_JOINT_FREE) { nq += 7; nv += 6; }
    else { nq += 1; nv += 1; nu += 1; }
  }
  for (int k = 0; k < nc; ++k) tp.clink[k] = clink[k];
  tp.nq = nq;
  tp.nv = nv;
  tp.nu = nu;
  tp.np = kParLink * n + kParSphere * nc;
  return tp;
}

template <typename R>
void rollout(const CTopo& tp, const double* Pd, const double* q0, const double* qd0, const double* tau, double dt,
             int T, double* traj, int* ncont, bool staged) {
  std::vector<R> stg(kStage);
  const PgsStage<R> stage{staged ? stg.data() : nullptr, 1};
  Art<R>* art = staged ? new Art<R> : nullptr;
  std::vector<R> Pv(Pd, Pd + tp.np);
  const Par<R> P{Pv.data(), 1, 0};
  const int nx = tp.nq + tp.nv;
  std::vector<R> x(nx), x1(nx), u(tp.nu > 0 ? tp.nu : 1);
  for (int k = 0; k < tp.nq; ++k) x[k] = R(q0[k]);
  for (int k = 0; k < tp.nv; ++k) x[tp.nq + k] = R(qd0[k]);
  for (int k = 0; k < nx; ++k) traj[k] = double(x[k]);
  auto* w = new Work<R>;
  for (int t = 0; t < T; ++t) {
    for (int k = 0; k < tp.nu; ++k) u[k] = R(tau[t * tp.nu + k]);
    ncont[t] = contact_step(tp, P, x.data(), x.data() + tp.nq, u.data(), R(dt), R(tp.mu), x1.data(),
                            x1.data() + tp.nq, *w, (Rec<R>*)nullptr, stage, art);
    x = x1;
    for (int k = 0; k < nx; ++k) traj[(t + 1) * nx + k] = double(x[k]);
  }
  delete w;
  delete art;
}

template <typename R>
void grad(const CTopo& tp, const double* Pd, const double* traj, const double* tau, double dt, int T,
          const double* gqT, const double* gqdT, double* gq0, double* gqd0, double* gtau, double* gmu) {
  using D = Dual<R>;
  std::vector<R> Pv(Pd, Pd + tp.np);
  const Par<R> P{Pv.data(), 1, 0};
  const int nq = tp.nq, nx = tp.nq + tp.nv, nu = tp.nu;
  std::vector<R> xb(nx), xn(nx);
  for (int k = 0; k < nq; ++k) xb[k] = R(gqT[k]);
  for (int k = 0; k < tp.nv; ++k) xb[nq + k] = R(gqdT[k]);
  auto* w = new Work<D>;
  std::vector<D> x(nx), x1(nx), u(nu > 0 ? nu : 1);
  R mu_acc = R(0);
  for (int t = T - 1; t >= 0; --t) {
    for (int j = 0; j < nx + nu + 1; ++j) {
      for (int k = 0; k < nx; ++k) x[k] = D(R(traj[t * nx + k]), R(k == j ? 1 : 0));
      for (int k = 0; k < nu; ++k) u[k] = D(R(tau[t * nu + k]), R(nx + k == j ? 1 : 0));
      contact_step(tp, P, x.data(), x.data() + nq, u.data(), R(dt), D(R(tp.mu), R(j == nx + nu ? 1 : 0)),
                   x1.data(), x1.data() + nq, *w);
      R s = R(0);
      for (int k = 0; k < nx; ++k) s += xb[k] * x1[k].d;
      if (j < nx) xn[j] = s;
      else if (j < nx + nu) gtau[t * nu + (j - nx)] = double(s);
      else mu_acc += s;
    }
    xb = xn;
  }
  delete w;
  for (int k = 0; k < nq; ++k) gq0[k] = double(xb[k]);
  for (int k = 0; k < tp.nv; ++k) gqd0[k] = double(xb[nq + k]);
  *gmu = double(mu_acc);
}

// the same gradient by the step's reverse statements (contact_step_vjp)
template <typename R>
void grad_adj(const CTopo& tp, const double* Pd, const double* traj, const double* tau, double dt, int T,
              const double* gqT, const double* gqdT, double* gq0, double* gqd0, double* gtau, double* gmu,
              bool staged) {
  std::vector<R> stg(kStage);
  const PgsStage<R> stage{staged ? stg.data() : nullptr, 1};
  std::vector<R> Pv(Pd, Pd + tp.np);
  const Par<R> P{Pv.data(), 1, 0};
  const int nq = tp.nq, nx = tp.nq + tp.nv, nu = tp.nu;
  std::vector<R> xb(nx), x(nx), u(nu > 0 ? nu : 1), ub(nu > 0 ? nu : 1);
  for (int k = 0; k < nq; ++k) xb[k] = R(gqT[k]);
  for (int k = 0; k < tp.nv; ++k) xb[nq + k] = R(gqdT[k]);
  auto* w = new Work<R>;
  auto* rc = new Rec<R>;
  auto* ad = new Adj<R>;
  auto* art = new Art<R>;
  R mu_acc = R(0);
  for (int t = T - 1; t >= 0; --t) {
    for (int k = 0; k < nx; ++k) x[k] = R(traj[t * nx + k]);
    for (int k = 0; k < nu; ++k) u[k] = R(tau[t * nu + k]);
    contact_step_vjp(tp, P, x.data(), x.data() + nq, u.data(), R(dt), R(tp.mu), xb.data(), ub.data(), mu_acc, *w,
                     *rc, *ad, *art, stage);
    for (int k = 0; k < nu; ++k) gtau[t * nu + k] = double(ub[k]);
  }
  delete w;
  delete rc;
  delete ad;
  delete art;
  for (int k = 0; k < nq; ++k) gq0[k] = double(xb[k]);
  for (int k = 0; k < tp.nv; ++k) gqd0[k] = double(xb[nq + k]);
  *gmu = double(mu_acc);
}

}  // namespace

extern "C" {

void emu_contact_grad_adj(int fp64, int n, const int* parent, const int* jtype, int nc, const int* clink, double mu,
                          double beta, int niter, const double* g, const double* P, const double* traj,
                          const double* tau, double dt, int T, const double* gqT, const double* gqdT, double* gq0,
                          double* gqd0, double* gtau, double* gmu, const double* limits, int staged) {
  const CTopo tp = topo(n, parent, jtype, nc, clink, mu, beta, niter, g, limits);
  if (fp64) grad_adj<double>(tp, P, traj, tau, dt, T, gqT, gqdT, gq0, gqd0, gtau, gmu, staged != 0);
  else grad_adj<float>(tp, P, traj, tau, dt, T, gqT, gqdT, gq0, gqd0, gtau, gmu, staged != 0);
}


// fp64 = 1: double arithmetic, 0: float (inputs and outputs are double either way)
void emu_contact_rollout(int fp64, int n, const int* parent, const int* jtype, int nc, const int* clink, double mu,
                         double beta, int niter, const double* g, const double* P, const double* q0,
                         const double* qd0, const double* tau, double dt, int T, double* traj, int* ncont,
                         const double* limits, int staged) {
  const CTopo tp = topo(n, parent, jtype, nc, clink, mu, beta, niter, g, limits);
  if (fp64) rollout<double>(tp, P, q0, qd0, tau, dt, T, traj, ncont, staged != 0);
  else rollout<float>(tp, P, q0, qd0, tau, dt, T, traj, ncont, staged != 0);
}

void emu_contact_grad(int fp64, int n, const int* parent, const int* jtype, int nc, const int* clink, double mu,
                      double beta, int niter, const double* g, const double* P, const double* traj,
                      const double* tau, double dt, int T, const double* gqT, const double* gqdT, double* gq0,
                      double* gqd0, double* gtau, double* gmu, const double* limits) {
  const CTopo tp = topo(n, parent, jtype, nc, clink, mu, beta, niter, g, limits);
  if (fp64) grad<double>(tp, P, traj, tau, dt, T, gqT, gqdT, gq0, gqd0, gtau, gmu);
  else grad<float>(tp, P, traj, tau, dt, T, gqT, gqdT, gq0, gqd0, gtau, gmu);
}

}  // extern "C"
