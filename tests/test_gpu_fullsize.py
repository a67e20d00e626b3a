"""GPU checks at the benchmark's full sizes and against central differences.

* The adjoint behind the autograd Function against central finite
  differences of the GPU's own FP64 rollout (torch.autograd.gradcheck): an
  oracle-free check of the whole differentiable path on chains, branched
  trees with prismatic joints and joint limits, and a free-floating
  quadruped (quaternion entries included).
* 8192 uneven trees x 2000 steps and 1024 quadrupeds x 50000 steps in the
  benchmark's launch configuration (autotuned geometry, one checkpoint per
  step).  As for the chains, long random-torque rollouts can be chaotic, so
  what is asserted holds at any horizon: on sampled systems the GPU's step
  map from its own states equals the oracle's step, and the GPU gradient
  equals the oracle's adjoint sweep along the GPU trajectory, for every
  checkpoint interval run (the quadrupeds' 1, 10 and 100).
* About 3 % of the quadrupeds' 50 s free falls diverge under semi-implicit
  Euler, in the FP64 oracle (14 of the first 512) as on the GPU in FP32 and
  FP64 (different systems: the rollouts are chaotic).  For such systems the
  test checks that the GPU follows the oracle's step map up to the
  divergence, so that what diverges is the method's integrator on this
  workload, not the kernels.
* Over 50 s the quadrupeds' exact gradients (FP64) grow to 1e40 - 1e70,
  beyond the FP32 range, because the adjoint of a chaotic rollout grows
  exponentially backward in time; the FP32 adjoint then overflows.  For such
  systems the control gradient of the final 500 steps is held to the FP32
  bar; over the final 2000 steps the figure is printed.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import TOL_GRAD_F32, rel
from paper_2109_07719_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _t(x, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


# ---------------------------------------------------------------- gradcheck

def _gradcheck_batch(T):
    draws = [synth.chain_system(4, 1500, T), synth.tree_system(2100, T, nmax=8, random_frames=True, prismatic=0.4),
             synth.quadruped_system(3100, T)]
    draws.append(synth.with_joint_limits(synth.chain_system(3, 1501, T), seed=7))
    return synth.make_batch(draws, 1e-3, name="gradcheck")


@pytest.mark.parametrize("K", [1, 3])
def test_autograd_adjoint_matches_central_differences_fp64(K):
    from paper_2109_07719_amd.sim import Sim, rollout
    b = _gradcheck_batch(12)
    sim = Sim(b.systems, b.gravity, dtype=torch.float64)
    q0 = _t(b.q0, torch.float64).requires_grad_()
    qd0 = _t(b.qd0, torch.float64).requires_grad_()
    tau = _t(b.tau, torch.float64).requires_grad_()
    w_q = torch.randn(q0.numel(), dtype=torch.float64, device=DEV, generator=torch.Generator(DEV).manual_seed(0))
    w_v = torch.randn(qd0.numel(), dtype=torch.float64, device=DEV, generator=torch.Generator(DEV).manual_seed(1))

    def f(a, c, u):
        qT, qdT = rollout(sim, a, c, u, b.dt, K=K)
        return (w_q * qT).sum() + (w_v * qdT).sum() + (qT ** 2).sum()

    assert torch.autograd.gradcheck(f, (q0, qd0, tau), eps=1e-6, atol=1e-7, rtol=1e-5)


# ---------------------------------------------------------------- full size

def _full_batch(name):
    b = synth.workload(name, tau_dtype=np.float32)
    r = synth.round_to_f32(synth.Batch(systems=b.systems, q0=b.q0, qd0=b.qd0, tau=b.tau[:1], dt=b.dt))
    return synth.Batch(systems=r.systems, q0=r.q0, qd0=r.qd0, tau=b.tau, dt=r.dt, gravity=r.gravity, name=b.name)


def _sampled_along(b, sample, K=1, extra_K=(), diverging=0):
    from paper_2109_07719_amd.sim import Sim
    sim = Sim(b.systems, b.gravity, dtype=torch.float32)
    tiling = sim.autotune(K=K, T_probe=min(b.T, 200))
    print("launch geometry", tiling)
    q0, qd0 = _t(b.q0), _t(b.qd0)
    tau = torch.from_numpy(b.tau).to(DEV)
    ws = sim.new_workspace(b.T, K)
    qT, qdT, tr = sim.forward(q0, qd0, tau, b.dt, K=K, workspace=ws, traj=True)
    seed_q, seed_v = 2 * qT, qdT.clone()
    gq0, gqd0, gtau = sim.backward(tau, b.dt, K, ws, seed_q, seed_v)
    status = sim.status()
    g_extra = []
    for K2 in extra_K:
        ws2 = sim.new_workspace(b.T, K2)
        sim.forward(q0, qd0, tau, b.dt, K=K2, workspace=ws2)
        g_extra.append([x.cpu().numpy() for x in sim.backward(tau, b.dt, K2, ws2, seed_q, seed_v)])
        del ws2
    del ws
    torch.cuda.synchronize()
    qo, vo, uo = b.offsets()
    nq = qo[-1]
    qTn, qdTn = qT.cpu().numpy(), qdT.cpu().numpy()
    diverged = [i for i in range(len(b.systems))
                if not (np.isfinite(qTn[qo[i]:qo[i + 1]]).all() and np.isfinite(qdTn[vo[i]:vo[i + 1]]).all())]
    print(f"{len(diverged)} of {len(b.systems)} systems diverged", diverged[:20])
    if not diverged:
        assert status == 0
    assert len(diverged) <= 0.1 * len(b.systems)
    import oracle as O
    worst_before = 0.0
    for i in diverged[:diverging]:
        # the GPU's step map equals the oracle's on the way to the divergence
        m = O.Model(b.systems[i], b.gravity)
        nqi = qo[i + 1] - qo[i]
        cols = np.r_[qo[i]:qo[i + 1], nq + vo[i]:nq + vo[i + 1]]
        traj_i = tr[:, torch.from_numpy(cols).to(DEV)].double().cpu().numpy()
        fin = np.isfinite(traj_i).all(axis=1)
        tb = int(np.argmin(fin))
        x0 = np.r_[b.q0[qo[i]:qo[i + 1]], b.qd0[vo[i]:vo[i + 1]]]
        states = np.concatenate([x0[None], traj_i[:-1]])
        tau_i = b.tau[:, uo[i]:uo[i + 1]].astype(np.float64)
        speeds = []
        for t in range(max(tb - 400, 0), tb - 10, 13):
            q1, qd1 = O.step(m, states[t, :nqi], states[t, nqi:], tau_i[t], b.dt)
            worst_before = max(worst_before, rel(traj_i[t], np.r_[q1, qd1]))
            speeds.append(np.abs(states[t, nqi:]).max())
        print(f"diverging system {i}: non-finite from step {tb}; step-map error on the way "
              f"{worst_before:.2e}, |qd| {min(speeds):.1e} .. {max(speeds):.1e}")
    assert worst_before < 1e-5
    sample = [i for i in sample if i not in diverged]
    gq0, gqd0 = gq0.cpu().numpy(), gqd0.cpu().numpy()
    gt_all = gtau.cpu().numpy()
    del gtau
    sq, sv = seed_q.cpu().numpy(), seed_v.cpu().numpy()
    assert sample
    rng = np.random.default_rng(0)
    worst_step, worst_grad, worst_window = 0.0, 0.0, 0.0
    for i in sample:
        m = O.Model(b.systems[i], b.gravity)
        nqi, nvi = qo[i + 1] - qo[i], vo[i + 1] - vo[i]
        cols = np.r_[qo[i]:qo[i + 1], nq + vo[i]:nq + vo[i + 1]]
        traj_i = tr[:, torch.from_numpy(cols).to(DEV)].double().cpu().numpy()
        x0 = np.r_[b.q0[qo[i]:qo[i + 1]], b.qd0[vo[i]:vo[i + 1]]]
        states = np.concatenate([x0[None], traj_i[:-1]])
        tau_i = b.tau[:, uo[i]:uo[i + 1]].astype(np.float64)
        for t in rng.choice(b.T, size=25, replace=False):
            q1, qd1 = O.step(m, states[t, :nqi], states[t, nqi:], tau_i[t], b.dt)
            worst_step = max(worst_step, rel(traj_i[t], np.r_[q1, qd1]))
        ga = O.adjoint_along(m, states, tau_i, b.dt, sq[qo[i]:qo[i + 1]], sv[vo[i]:vo[i + 1]])
        # the exact gradient of a long chaotic rollout can exceed the FP32 range
        # (it grows exponentially backward in time); then only the control
        # gradient of the final steps is representable and compared
        size = max(np.abs(x).max() for x in ga[:3] if x.size)
        fits = size < 1e-3 * float(np.finfo(np.float32).max)
        W = b.T if fits else min(b.T, 500)
        # a ball joint's quaternion gradient is compared along the unit sphere
        ga0 = O.ball_tangent(b.systems[i], x0[:nqi], ga[0])
        for K2, g in [(K, (gq0, gqd0, gt_all))] + list(zip(extra_K, g_extra)):
            gt_i = g[2][-W:, uo[i]:uo[i + 1]]
            e = [rel(gt_i, ga[2][-W:])] if gt_i.size else []
            if fits:
                e += [rel(g[0][qo[i]:qo[i + 1]], ga0), rel(g[1][vo[i]:vo[i + 1]], ga[1])]
            if fits:
                worst_grad = max(worst_grad, *e)
            else:
                worst_window = max(worst_window, *e)
            note = ""
            if not fits:
                note = " (last 2000 steps: %.1e)" % rel(g[2][-2000:, uo[i]:uo[i + 1]], ga[2][-2000:])
            print("system", i, f"({nvi} DOF), K={K2}:", "gradient error along the GPU trajectory" if fits else
                  f"exact gradient {size:.1e} beyond FP32; control-gradient error over the last {W} steps",
                  ["%.1e" % x for x in e], note)
    print(f"worst step-map error {worst_step:.2e}, worst gradient error along trajectory {worst_grad:.2e}, "
          f"worst final-window control-gradient error {worst_window:.2e}")
    return worst_step, worst_grad, worst_window


def test_full_size_trees_8192_sampled():
    b = _full_batch("trees_8192")
    assert len(b.systems) == 8192 and b.T == 2000
    sample = [0, 1, 777, 4096, 6000, 8191]
    worst_step, worst_grad, worst_window = _sampled_along(b, sample)
    assert worst_step < 1e-6
    assert worst_grad < TOL_GRAD_F32 and worst_window == 0.0


def test_full_size_ball_quadrupeds_1024_sampled():
    """1024 quadrupeds on ball hips, 2000 steps (11 rollouts diverge under
    the integrator, the FP64 oracle's the same 11): sampled step maps and
    gradients along the GPU trajectory, K = 1 and 10."""
    b = _full_batch("ball_quad_1024")
    assert len(b.systems) == 1024 and b.T == 2000
    worst_step, worst_grad, worst_window = _sampled_along(b, [0, 300, 511, 777, 1023], extra_K=(10,), diverging=0)
    assert worst_step < 1e-6
    assert worst_grad < TOL_GRAD_F32 and worst_window == 0.0


def test_full_size_quadrupeds_1024_sampled():
    b = _full_batch("quad_1024")
    assert len(b.systems) == 1024 and b.T == 50000
    worst_step, worst_grad, worst_window = _sampled_along(b, [0, 511, 1023], extra_K=(10, 100), diverging=2)
    assert worst_step < 1e-6
    assert worst_grad < TOL_GRAD_F32
    # the final 0.5 s of control gradients, at the 450-490 m/s body-frame base
    # speed that 50 s of free fall reaches, hold the FP32 bar
    assert worst_window < TOL_GRAD_F32
