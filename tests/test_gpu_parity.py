"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Errors are per system and norm-wise (||x - ref|| / max(||ref||, floor)).
Bars (FP32): forward dynamics 1e-5 per step from identical input states,
state 1e-3 after 1000 steps, gradients 1e-3; FP64 handles are held to
round-off.  Every input is seeded and synthetic; the oracle sees the same
FP32-rounded values widened to FP64.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import (FLOOR_F64, TOL_GRAD_F32, TOL_QDD_F32, TOL_STATE_F32, oracle_fd, oracle_grads, rel)
from paper_2109_07719_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _sim(batch, dtype=torch.float32, adj=None):
    """adj: the reverse passes' arithmetic of an FP32 handle ("f64", the
    default, or "f32")."""
    from paper_2109_07719_amd.sim import Sim
    sim = Sim(batch.systems, batch.gravity, dtype=dtype)
    if adj is not None:
        sim.set_adjoint_dtype(torch.float64 if adj == "f64" else torch.float32)
    return sim


def _t(x, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def _batch(name, n, T, f32=True):
    b = synth.workload(name, n_systems=n, T=T)
    return synth.round_to_f32(b) if f32 else b


def _mixed_batch(T, seed=0):
    """Chains, uneven trees and quadrupeds in one handle (ragged packing)."""
    draws = [synth.chain_system(7, 1000 + i, T) for i in range(5)]
    draws += [synth.tree_system(2000 + i, T, random_frames=(i % 2 == 1)) for i in range(9)]
    draws += [synth.quadruped_system(3000 + i, T) for i in range(3)]
    draws += [synth.chain_system(n, 4000 + n, T) for n in (1, 2, 64)]
    return synth.round_to_f32(synth.make_batch(draws, 1e-3, name="mixed"))


def _random_state(batch, rng):
    """Random states (unit quaternions for free roots) for single-step checks."""
    qo, vo, uo = batch.offsets()
    q = rng.normal(0, 0.5, qo[-1])
    for i, s in enumerate(batch.systems):
        if s.jtype[0] == 1:
            qt = rng.normal(size=4)
            q[qo[i] + 3:qo[i] + 7] = qt / np.linalg.norm(qt)
    qd = rng.normal(0, 0.5, vo[-1])
    tau = rng.normal(0, 1, uo[-1])
    r = lambda x: x.astype(np.float32).astype(np.float64)
    return r(q), r(qd), r(tau)


# ------------------------------------------------------------- forward dynamics

@pytest.mark.parametrize("name,n", [("chain7_4096", 64), ("trees_8192", 48), ("quad_1024", 16)])
def test_aba_qdd_fp32(name, n):
    b = _batch(name, n, 1)
    sim = _sim(b)
    rng = np.random.default_rng(7)
    q, qd, tau = _random_state(b, rng)
    qdd = sim.aba(_t(q), _t(qd), _t(tau)).cpu().numpy()
    ref = oracle_fd(b, q, qd, tau)
    vo = b.offsets()[1]
    errs = [rel(qdd[vo[i]:vo[i + 1]], ref[i]) for i in range(n)]
    print(f"{name}: qdd rel err max {max(errs):.2e} median {np.median(errs):.2e}")
    assert max(errs) < TOL_QDD_F32


def test_aba_qdd_fp64_mixed():
    b = _mixed_batch(1)
    sim = _sim(b, torch.float64)
    q, qd, tau = _random_state(b, np.random.default_rng(3))
    qdd = sim.aba(_t(q, torch.float64), _t(qd, torch.float64), _t(tau, torch.float64)).cpu().numpy()
    ref = oracle_fd(b, q, qd, tau)
    vo = b.offsets()[1]
    errs = [rel(qdd[vo[i]:vo[i + 1]], ref[i], FLOOR_F64) for i in range(len(b.systems))]
    assert max(errs) < 1e-11, errs


def test_fast_free_base_fp32():
    """A free base moving at 300 and 3000 m/s (what a long free fall
    reaches): the kernels' Galilean shift of the root keeps FP32 joint and
    base accelerations within the forward-dynamics bar."""
    draws = [synth.quadruped_system(3000 + i, 1) for i in range(6)]
    b = synth.round_to_f32(synth.make_batch(draws, 1e-3))
    sim = _sim(b)
    qo, vo, uo = b.offsets()
    for speed in (300.0, 3000.0):
        q, qd, tau = _random_state(b, np.random.default_rng(int(speed)))
        rng = np.random.default_rng(7)
        for i in range(len(b.systems)):
            d = rng.normal(size=3)
            qd[vo[i] + 3:vo[i] + 6] = speed * d / np.linalg.norm(d)
        qd = qd.astype(np.float32).astype(np.float64)
        got = sim.aba(_t(q), _t(qd), _t(tau)).cpu().numpy()
        ref = oracle_fd(b, q, qd, tau)
        # joints and base separately: the base's linear acceleration carries
        # the large w x v_lin term
        errs = [max(rel(got[vo[i] + 6:vo[i + 1]], ref[i][6:], 1e-6), rel(got[vo[i]:vo[i] + 6], ref[i][:6], 1e-6))
                for i in range(len(b.systems))]
        print(speed, "m/s:", ["%.1e" % e for e in errs])
        assert max(errs) < TOL_QDD_F32


def test_aba_qdd_fp32_mixed_ragged():
    b = _mixed_batch(1)
    sim = _sim(b)
    assert sim.info["n_waves"] > 1
    q, qd, tau = _random_state(b, np.random.default_rng(4))
    q, qd = q * 0.2, qd * 0.2
    q, qd = q.astype(np.float32).astype(np.float64), qd.astype(np.float32).astype(np.float64)
    # keep free-root quaternions unit
    qo = b.offsets()[0]
    for i, s in enumerate(b.systems):
        if s.jtype[0] == 1:
            q[qo[i] + 3:qo[i] + 7] = [0, 0, 0, 1]
    qdd = sim.aba(_t(q), _t(qd), _t(tau)).cpu().numpy()
    ref = oracle_fd(b, q, qd, tau)
    vo = b.offsets()[1]
    errs = [rel(qdd[vo[i]:vo[i + 1]], ref[i]) for i in range(len(b.systems))]
    print("mixed qdd errs", ["%.1e" % e for e in errs])
    # the 64-link chain is ill-conditioned in FP32; every other system meets the bar
    n64 = len(b.systems) - 1
    assert max(e for i, e in enumerate(errs) if i != n64) < TOL_QDD_F32
    assert errs[n64] < 1e-3


# ------------------------------------------------------------- rollouts

def _rollout(sim, b, K=1, traj=False, dtype=torch.float32):
    q0, qd0, tau = _t(b.q0, dtype), _t(b.qd0, dtype), _t(b.tau, dtype)
    ws = sim.new_workspace(b.T, K)
    qT, qdT, tr = sim.forward(q0, qd0, tau, b.dt, K=K, workspace=ws, traj=traj)
    return q0, qd0, tau, ws, qT, qdT, tr


def test_state_after_1000_steps_chain7_fp32():
    b = _batch("chain7_4096", 64, 1000)
    sim = _sim(b)
    _, _, _, _, qT, qdT, _ = _rollout(sim, b)
    qT, qdT = qT.cpu().numpy(), qdT.cpu().numpy()
    ref = oracle_grads(b, lambda i, q, v: (np.zeros_like(q), np.zeros_like(v)))
    qo, vo, _ = b.offsets()
    errs = [rel(np.r_[qT[qo[i]:qo[i + 1]], qdT[vo[i]:vo[i + 1]]], np.r_[ref[i][3], ref[i][4]])
            for i in range(64)]
    print(f"state after 1000 steps: max {max(errs):.2e}")
    assert max(errs) < TOL_STATE_F32


def _grad_parity(b, K=1, tol=TOL_GRAD_F32, dtype=torch.float32, floor=1e-6, with_traj=False, adj=None):
    sim = _sim(b, dtype, adj)
    q0, qd0, tau, ws, qT, qdT, tr = _rollout(sim, b, K=K, traj=with_traj, dtype=dtype)
    rng = np.random.default_rng(5)
    qo, vo, uo = b.offsets()
    gtraj_np = rng.normal(size=(b.T, b.offsets()[0][-1] + b.offsets()[1][-1])) * 1e-3 if with_traj else None
    gqT = 2 * qT
    gqdT = torch.zeros_like(qdT)
    gq0, gqd0, gtau = sim.backward(tau, b.dt, K, ws, gqT, gqdT,
                                   _t(gtraj_np, dtype) if with_traj else None)
    gq0, gqd0, gtau = gq0.cpu().numpy(), gqd0.cpu().numpy(), gtau.cpu().numpy()
    nq = qo[-1]
    gtr = None
    if with_traj:
        gtr = [np.concatenate([gtraj_np[:, qo[i]:qo[i + 1]], gtraj_np[:, nq + vo[i]:nq + vo[i + 1]]], axis=1)
               for i in range(len(b.systems))]
    ref = oracle_grads(b, lambda i, q, v: (2 * q, np.zeros_like(v)), gtraj=gtr)
    worst = {}
    for i in range(len(b.systems)):
        r = ref[i]
        for nm, x, y in (("gq0", gq0[qo[i]:qo[i + 1]], r[0]), ("gqd0", gqd0[vo[i]:vo[i + 1]], r[1]),
                         ("gtau", gtau[:, uo[i]:uo[i + 1]], r[2])):
            worst[nm] = max(worst.get(nm, 0.0), rel(x, y, floor))
    print(b.name, "K", K, "adjoint", adj or "default", {k: "%.2e" % v for k, v in worst.items()})
    assert max(worst.values()) < tol, worst
    return gq0, gqd0, gtau


# FP32 handles: the reverse passes in FP64 (default) and in FP32.  With the
# FP64 reverse the FP32 tape's rounding is what remains, so its bar is held
# ten times tighter than the FP32 gradient bar.
ADJ = [("f64", TOL_GRAD_F32 / 10), ("f32", TOL_GRAD_F32)]


@pytest.mark.parametrize("adj,tol", ADJ)
def test_gradients_chain7_fp32_1000_steps(adj, tol):
    _grad_parity(_batch("chain7_4096", 64, 1000), adj=adj, tol=tol)


@pytest.mark.parametrize("adj,tol", ADJ)
def test_gradients_chain7_fp32_with_traj_seed(adj, tol):
    _grad_parity(_batch("chain7_4096", 16, 300), with_traj=True, adj=adj, tol=tol)


@pytest.mark.parametrize("adj,tol", ADJ)
def test_gradients_trees_fp32(adj, tol):
    _grad_parity(_batch("trees_8192", 24, 400), adj=adj, tol=tol)


@pytest.mark.parametrize("adj,tol", ADJ)
def test_gradients_quadruped_fp32(adj, tol):
    _grad_parity(_batch("quad_1024", 8, 500), adj=adj, tol=tol)


def test_gradients_chain7_fp64_config():
    """The single 7-link chain in FP64, 1000 steps, L = sum q_T^2."""
    b = _batch("chain7_fp64", 1, 1000, f32=False)
    _grad_parity(b, tol=1e-9, dtype=torch.float64, floor=FLOOR_F64)


def test_gradients_mixed_fp64_round_off():
    b = synth.make_batch([synth.chain_system(7, 1000, 300), synth.tree_system(2001, 300, random_frames=True),
                          synth.quadruped_system(3001, 300)], 1e-3, name="mixed64")
    _grad_parity(b, tol=1e-9, dtype=torch.float64, floor=FLOOR_F64, with_traj=True)


@pytest.mark.parametrize("adj", ["f64", "f32"])
@pytest.mark.parametrize("K", [3, 10, 100])
def test_checkpoint_interval_matches_K1(K, adj):
    b = _batch("chain7_4096", 32, 250)
    g1 = _grad_parity(b, K=1, adj=adj)
    gk = _grad_parity(b, K=K, adj=adj)
    for a, c in zip(g1, gk):
        assert np.allclose(a, c, rtol=1e-4, atol=1e-6)
    print("K", K, "bitwise equal to K=1:", all(np.array_equal(a, c) for a, c in zip(g1, gk)))


@pytest.mark.parametrize("adj", ["f64", "f32"])
@pytest.mark.parametrize("name,n,T", [("chain7_4096", 32, 250), ("quad_1024", 4, 120), ("trees_8192", 6, 90)])
def test_store_all_matches_recompute(name, n, T, adj):
    """Store-all (every step's intermediates kept, no recompute) gives the
    same gradients as per-step checkpoints with recompute."""
    b = _batch(name, n, T)
    g1 = _grad_parity(b, K=1, adj=adj)
    g0 = _grad_parity(b, K=0, adj=adj)
    for a, c in zip(g1, g0):
        assert np.allclose(a, c, rtol=1e-5, atol=1e-7)
    print(name, "store-all bitwise equal to K=1:", all(np.array_equal(a, c) for a, c in zip(g1, g0)))


def test_store_all_workspace_is_larger():
    b = _batch("quad_1024", 4, 100)
    sim = _sim(b)
    w0, w1, w10 = sim.workspace_bytes(100, 0), sim.workspace_bytes(100, 1), sim.workspace_bytes(100, 10)
    assert w0 > 20 * w1 > 20 * w10 / 10


def test_quadruped_checkpoint_interval():
    b = _batch("quad_1024", 4, 120)
    g1 = _grad_parity(b, K=1)
    g7 = _grad_parity(b, K=7)
    for a, c in zip(g1, g7):
        assert np.allclose(a, c, rtol=1e-4, atol=1e-6)


def test_batch_independence_and_determinism():
    """A system's results do not depend on what else is in the batch, and
    repeated runs are bitwise equal."""
    big = _batch("chain7_4096", 40, 200)
    small = synth.round_to_f32(synth.make_batch([synth.chain_system(7, 1000 + i, 200) for i in range(5)], 1e-3))
    outs = []
    for b in (big, big, small):
        sim = _sim(b)
        q0, qd0, tau, ws, qT, qdT, _ = _rollout(sim, b)
        g = sim.backward(tau, b.dt, 1, ws, 2 * qT, torch.zeros_like(qdT))
        outs.append([qT.cpu().numpy(), g[0].cpu().numpy(), g[2].cpu().numpy()])
    for a, c in zip(outs[0], outs[1]):
        assert np.array_equal(a, c)
    assert np.array_equal(outs[0][0][:35], outs[2][0])
    assert np.array_equal(outs[0][1][:35], outs[2][1])
    assert np.array_equal(outs[0][2][:, :35], outs[2][2])


def test_traj_output_matches_stepwise_oracle():
    b = _batch("quad_1024", 3, 50)
    sim = _sim(b)
    _, _, _, _, qT, qdT, tr = _rollout(sim, b, traj=True)
    import oracle as O
    tr = tr.cpu().numpy()
    qo, vo, uo = b.offsets()
    nq = qo[-1]
    for i, s in enumerate(b.systems):
        m = O.Model(s, b.gravity)
        _, _, ref = O.rollout(m, b.q0[qo[i]:qo[i + 1]], b.qd0[vo[i]:vo[i + 1]], b.tau[:, uo[i]:uo[i + 1]],
                              b.dt, traj=True)
        mine = np.concatenate([tr[:, qo[i]:qo[i + 1]], tr[:, nq + vo[i]:nq + vo[i + 1]]], axis=1)
        assert rel(mine, ref) < 1e-4
    assert np.array_equal(tr[-1, :nq], qT.cpu().numpy())


def test_autograd_function_matches_direct_calls():
    from paper_2109_07719_amd.sim import rollout
    b = _batch("trees_8192", 6, 100)
    sim = _sim(b)
    q0 = _t(b.q0).requires_grad_()
    qd0 = _t(b.qd0).requires_grad_()
    tau = _t(b.tau).requires_grad_()
    qT, qdT, tr = rollout(sim, q0, qd0, tau, b.dt, K=4, traj=True)
    loss = (qT ** 2).sum() + 0.5 * (qdT ** 2).sum() + (tr[::7] ** 2).sum() * 1e-2
    loss.backward()
    # direct: seeds formed by hand
    ws = sim.new_workspace(b.T, 4)
    qT2, qdT2, tr2 = sim.forward(q0.detach(), qd0.detach(), tau.detach(), b.dt, K=4, workspace=ws, traj=True)
    gtr = torch.zeros_like(tr2)
    gtr[::7] = 2e-2 * tr2[::7]
    g = sim.backward(tau.detach(), b.dt, 4, ws, 2 * qT2, qdT2, gtr)
    assert torch.equal(g[0], q0.grad) and torch.equal(g[1], qd0.grad) and torch.equal(g[2], tau.grad)


# ------------------------------------------------------------- edge cases

def test_zero_and_one_step():
    b = _batch("chain7_4096", 3, 1)
    sim = _sim(b)
    q0, qd0, tau = _t(b.q0), _t(b.qd0), _t(b.tau)
    qT, qdT, _ = sim.forward(q0, qd0, tau[:0], b.dt, K=1, workspace=sim.new_workspace(0, 1))
    assert torch.equal(qT, q0) and torch.equal(qdT, qd0)
    g = sim.backward(tau[:0], b.dt, 1, sim.new_workspace(0, 1), qT, qdT)
    assert torch.equal(g[0], qT) and torch.equal(g[1], qdT) and g[2].numel() == 0
    _grad_parity(b)


def test_free_body_without_joints():
    """A lone free-floating body (nu = 0): ballistic flight with rotation."""
    s = synth.System(parent=np.array([-1], np.int32), jtype=np.array([1], np.int32),
                     E_T=np.eye(3)[None], r_T=np.zeros((1, 3)), axis=np.array([[0, 0, 1.0]]),
                     mass=np.array([2.0]), com=np.array([[0.1, 0.0, 0.0]]),
                     Ic=np.array([[0.1, 0.2, 0.3, 0.0, 0.0, 0.0]]))
    q0 = np.array([0, 0, 0, 0, 0, 0, 1.0])
    qd0 = np.array([0.3, -0.2, 0.5, 1.0, 2.0, 0.0])
    b = synth.round_to_f32(synth.make_batch([(s, q0, qd0, np.zeros((200, 0)))], 1e-3))
    _grad_parity(b)


def test_invalid_calls_raise():
    from paper_2109_07719_amd._native import SimError
    b = _batch("chain7_4096", 2, 10)
    sim = _sim(b)
    q0, qd0, tau = _t(b.q0), _t(b.qd0), _t(b.tau)
    with pytest.raises(SimError):
        sim.forward(q0, qd0, tau, -1.0)
    with pytest.raises(SimError):
        sim.forward(q0, qd0, tau, b.dt, K=-5000)   # K < 0 is binomial checkpointing with at most 4096 snapshots
    small = torch.empty(8, dtype=torch.uint8, device=DEV)
    with pytest.raises(SimError):
        sim.forward(q0, qd0, tau, b.dt, K=1, workspace=small)


def test_closed_handle_fails_cleanly():
    """close() releases the handle once; later calls report an error
    instead of touching freed memory, and many short-lived handles leave the
    library in a working state."""
    from paper_2109_07719_amd._native import SimError
    b = _batch("chain7_4096", 2, 10)
    for _ in range(20):
        _sim(b)
    sim = _sim(b)
    q0, qd0, tau = _t(b.q0), _t(b.qd0), _t(b.tau)
    qT, _, _ = sim.forward(q0, qd0, tau, b.dt)
    sim.close()
    sim.close()
    with pytest.raises(SimError):
        sim.forward(q0, qd0, tau, b.dt)
    qT2, _, _ = _sim(b).forward(q0, qd0, tau, b.dt)
    assert torch.equal(qT, qT2)


# ------------------------------------------------------------- full size

def test_full_size_chain7_4096_sampled():
    """4096 chains x 5000 steps in the benchmark's launch configuration.
    Over 5 s of random torques some chains are chaotic (a 1e-7 change of q0
    moves q_T by tens of percent even in FP64), so the end-to-end FP32-vs-
    FP64 difference is reported, not asserted.  What holds at any horizon is
    checked on sampled systems: (1) the GPU's step map from its own states
    equals the oracle's step; (2) the GPU gradient equals the oracle's
    adjoint sweep along the GPU trajectory (its states used as the per-step
    checkpoints)."""
    import oracle as O
    b = synth.workload("chain7_4096", T=5000, tau_dtype=np.float32)
    r = synth.round_to_f32(synth.Batch(systems=b.systems, q0=b.q0, qd0=b.qd0, tau=b.tau[:1], dt=b.dt))
    b = synth.Batch(systems=r.systems, q0=r.q0, qd0=r.qd0, tau=b.tau, dt=r.dt, gravity=r.gravity, name=b.name)
    sim = _sim(b)
    q0, qd0 = _t(b.q0), _t(b.qd0)
    tau = torch.from_numpy(b.tau).to(DEV)
    ws = sim.new_workspace(b.T, 1)
    qT, qdT, tr = sim.forward(q0, qd0, tau, b.dt, K=1, workspace=ws, traj=True)
    gq0, gqd0, gtau = sim.backward(tau, b.dt, 1, ws, 2 * qT, torch.zeros_like(qdT))
    torch.cuda.synchronize()
    qo, vo, uo = b.offsets()
    nq = qo[-1]
    sample = [0, 1, 1234, 2047, 3000, 4095]
    gq0, gqd0, gtau, qTn = gq0.cpu().numpy(), gqd0.cpu().numpy(), gtau.cpu().numpy(), qT.cpu().numpy()
    rng = np.random.default_rng(0)
    worst_step, worst_grad = 0.0, 0.0
    for i in sample:
        m = O.Model(b.systems[i], b.gravity)
        cols = np.r_[qo[i]:qo[i + 1], nq + vo[i]:nq + vo[i + 1]]
        traj_i = tr[:, torch.from_numpy(cols).to(DEV)].double().cpu().numpy()
        x0 = np.r_[b.q0[qo[i]:qo[i + 1]], b.qd0[vo[i]:vo[i + 1]]]
        states = np.concatenate([x0[None], traj_i[:-1]])
        tau_i = b.tau[:, uo[i]:uo[i + 1]].astype(np.float64)
        for t in rng.choice(b.T, size=25, replace=False):
            q1, qd1 = O.step(m, states[t, :7], states[t, 7:], tau_i[t], b.dt)
            worst_step = max(worst_step, rel(traj_i[t], np.r_[q1, qd1]))
        ga = O.adjoint_along(m, states, tau_i, b.dt, 2 * traj_i[-1, :7], np.zeros(7))
        e_along = [rel(gq0[qo[i]:qo[i + 1]], ga[0]), rel(gqd0[vo[i]:vo[i + 1]], ga[1]),
                   rel(gtau[:, uo[i]:uo[i + 1]], ga[2])]
        worst_grad = max(worst_grad, *e_along)
        ref = O.rollout_grad(m, x0[:7], x0[7:], tau_i, b.dt,
                             2 * O.rollout(m, x0[:7], x0[7:], tau_i, b.dt)[0], np.zeros(7))
        e2e = [rel(qTn[qo[i]:qo[i + 1]], ref[3]), rel(gq0[qo[i]:qo[i + 1]], ref[0]),
               rel(gtau[:, uo[i]:uo[i + 1]], ref[2])]
        print("system", i, "grad along GPU trajectory", ["%.1e" % x for x in e_along],
              "| end-to-end vs FP64 (qT, gq0, gtau)", ["%.1e" % x for x in e2e])
    print(f"worst step-map error {worst_step:.2e}, worst gradient error along trajectory {worst_grad:.2e}")
    assert np.all(np.isfinite(gtau))
    assert worst_step < 1e-6
    assert worst_grad < TOL_GRAD_F32


def test_trajectory_optimisation_gradients_match_fp64_oracle():
    """Trajectory optimisation (end-effector target + 1e-4 ||tau||^2, Adam):
    the gradient the autograd Function hands to the optimiser equals the FP64
    oracle's (torch FP64 forward kinematics for the seed, oracle adjoint for
    dL/dtau) at several iterations."""
    import oracle as O
    from paper_2109_07719_amd.fk import LinkPoints
    from paper_2109_07719_amd.trajopt import TrajOpt, chains_problem
    b, targets = chains_problem(n_systems=48, T=200)
    opt = TrajOpt(b, targets, [s.n - 1 for s in b.systems], np.tile([0.5, 0, 0], (48, 1)))
    qo, vo, uo = b.offsets()
    check = [0, 5, 17, 30, 47]
    losses = []
    for it in range(12):
        opt.opt.zero_grad()
        L, _ = opt.loss()
        L.backward()
        losses.append(float(L.detach()))
        if it in (0, 6, 11):
            tau = opt.tau.detach().double().cpu().numpy()
            g = opt.tau.grad.detach().cpu().numpy()
            for i in check:
                s = b.systems[i]
                m = O.Model(s, b.gravity)
                ti = tau[:, uo[i]:uo[i + 1]]
                qT, qdT = O.rollout(m, b.q0[qo[i]:qo[i + 1]], b.qd0[vo[i]:vo[i + 1]], ti, b.dt)
                fk = LinkPoints([s], [s.n - 1], [[0.5, 0, 0]], dtype=torch.float64, device="cpu")
                qt = torch.tensor(qT, requires_grad=True)
                ((fk(qt) - torch.tensor(targets[i:i + 1])) ** 2).sum().backward()
                ref = O.rollout_grad(m, b.q0[qo[i]:qo[i + 1]], b.qd0[vo[i]:vo[i + 1]], ti, b.dt,
                                     qt.grad.numpy(), np.zeros(s.nv))
                ref_tau = ref[2] + 2e-4 * ti
                e = rel(g[:, uo[i]:uo[i + 1]], ref_tau)
                print(f"iter {it} chain {i} (n={s.n}) grad rel err {e:.2e}")
                assert e < TOL_GRAD_F32
        opt.opt.step()
    print("loss", ["%.3g" % x for x in losses])
    assert losses[-1] < losses[0]


@pytest.mark.parametrize("kind", ["mixed", "chains"])
def test_launch_geometry_changes_no_arithmetic(kind):
    """Every launch geometry (wavefronts per workgroup, producer/consumer
    pairs per workgroup, pipelined or one-wave adjoint) gives bitwise the
    same rollout, gradients and forward dynamics."""
    if kind == "mixed":
        b = _mixed_batch(60)
    else:
        b = synth.round_to_f32(synth.make_batch([synth.chain_system(n, 6000 + n, 60) for n in (1, 3, 7, 7, 9, 30)],
                                                1e-3))
    sim = _sim(b)
    q, qd, tau1 = _random_state(b, np.random.default_rng(9))
    results = {}
    for tl in [(1, 1, 1), (2, 1, 1), (4, 2, 1), (4, 1, 0), (2, 2, 1)]:
        sim.set_tiling(*tl)
        assert sim.tiling == dict(zip(("waves_per_block", "pairs_per_block", "pipelined"), tl))
        out = []
        for K in (1, 3):
            q0, qd0, tau, ws, qT, qdT, _ = _rollout(sim, b, K=K)
            g = sim.backward(tau, b.dt, K, ws, 2 * qT, torch.zeros_like(qdT))
            out += [x.cpu().numpy() for x in (qT, qdT, *g)]
        out.append(sim.aba(_t(q), _t(qd), _t(tau1)).cpu().numpy())
        results[tl] = out
    ref = results[(1, 1, 1)]
    for tl, out in results.items():
        for j, (a, c) in enumerate(zip(ref, out)):
            if tl[2] == 0 and j < 5:
                # K = 1 without the pipelined kernel: the reverse passes read
                # the recomputed intermediates from registers instead of the
                # LDS tape, so the compiler may contract differently
                assert rel(c, a) < 1e-5, tl
            else:
                assert np.array_equal(a, c), tl
    with pytest.raises(Exception):
        sim.set_tiling(3, 1, 1)
    with pytest.raises(Exception):
        sim.set_tiling(1, 4, 1)


@pytest.mark.parametrize("K", [1, 0, 5])
def test_autotune_keeps_a_valid_geometry_and_the_results(K):
    b = _mixed_batch(40)
    sim = _sim(b)
    out0 = None
    for phase in range(2):
        if phase == 1:
            t = sim.autotune(K=K, T_probe=30)
            assert t["waves_per_block"] in (1, 2, 4) and t["pairs_per_block"] in (1, 2) and t["pipelined"] in (0, 1)
            assert t["ms_per_probe_step"] > 0
            assert {k: t[k] for k in sim.tiling} == sim.tiling
        q0, qd0, tau, ws, qT, qdT, _ = _rollout(sim, b, K=K)
        g = sim.backward(tau, b.dt, K, ws, 2 * qT, torch.zeros_like(qdT))
        out = [x.cpu().numpy() for x in (qT, qdT, *g)]
        if out0 is None:
            out0 = out
    for a, c in zip(out0, out):
        assert rel(c, a) < 1e-5
    with pytest.raises(Exception):
        sim.autotune(K=-5000)
    with pytest.raises(Exception):
        sim.autotune(K=1, T_probe=0)


def test_autotune_choices_are_kept_per_structure():
    """A second handle of the same structure gets the first one's choice
    without probing (the same ms per probe step, bit for bit); another
    structure, another adjoint dtype or a cleared cache probes again."""
    from paper_2109_07719_amd import _native as N
    N.lib().sim_autotune_cache_clear()
    b = _mixed_batch(40)
    s1, s2 = _sim(b), _sim(b)
    t1 = s1.autotune(K=1, T_probe=30)
    t2 = s2.autotune(K=1, T_probe=30)
    assert t2 == t1
    t3 = _sim(b, adj="f32").autotune(K=1, T_probe=30)
    chains = synth.round_to_f32(synth.make_batch([synth.chain_system(7, 1000 + i, 40) for i in range(6)], 1e-3,
                                                 name="chains"))
    t4 = _sim(chains).autotune(K=1, T_probe=30)
    t5 = s1.autotune(K=5, T_probe=30)
    assert len({t1["ms_per_probe_step"], t3["ms_per_probe_step"], t4["ms_per_probe_step"],
                t5["ms_per_probe_step"]}) == 4
    N.lib().sim_autotune_cache_clear()
    t6 = s2.autotune(K=1, T_probe=30)
    assert t6["ms_per_probe_step"] != t1["ms_per_probe_step"]


def test_status_counts_nonfinite_outputs():
    b = _mixed_batch(50)
    sim = _sim(b)
    assert sim.status() == 0
    q0, qd0, tau, ws, qT, qdT, _ = _rollout(sim, b)
    sim.backward(tau, b.dt, 1, ws, 2 * qT, torch.zeros_like(qdT))
    assert sim.status() == 0
    # a NaN torque at step 20 of one chain poisons that chain's final state
    # and its gradients, and nothing else
    tau_bad = tau.clone()
    tau_bad[20, 0] = float("nan")
    qT2, qdT2, _ = sim.forward(q0, qd0, tau_bad, b.dt, K=1, workspace=ws)
    n_fwd = sim.status()
    s0 = b.systems[0]
    assert n_fwd == s0.nq + s0.nv
    assert torch.isfinite(qT2[s0.nq:]).all() and torch.isfinite(qdT2[s0.nv:]).all()
    sim.backward(tau_bad, b.dt, 1, ws, torch.zeros_like(qT2), torch.zeros_like(qdT2))
    assert sim.status() > 0
    assert sim.status() == 0
    qd_bad = qd0.clone()
    qd_bad[1] = float("inf")
    sim.aba(q0, qd_bad, tau[0].contiguous())
    assert sim.status() > 0


@pytest.mark.parametrize("s", [1, 3, 8])
@pytest.mark.parametrize("kind", ["mixed", "chains"])
def test_binomial_checkpointing_matches_uniform_checkpoints(kind, s):
    """K = -s (binomial schedule, s snapshots) repeats the same step
    arithmetic as segment replay, so gradients (and parameter gradients)
    are bitwise those of K = 3 on the same one-wave kernel."""
    if kind == "mixed":
        b = _mixed_batch(70)
    else:
        b = synth.round_to_f32(synth.make_batch([synth.chain_system(n, 6100 + n, 70) for n in (1, 4, 7, 12)], 1e-3))
    sim = _sim(b)
    sim.set_tiling(4, 1, 0)
    outs = []
    for K in (3, -s):
        q0, qd0, tau, ws, qT, qdT, _ = _rollout(sim, b, K=K)
        g = sim.backward(tau, b.dt, K, ws, 2 * qT, torch.zeros_like(qdT), params=True)
        outs.append([x.cpu().numpy() for x in (qT, qdT, *g)])
        assert sim.status() == 0
    for a, c in zip(*outs):
        assert np.array_equal(a, c)
    assert sim.workspace_bytes(70, -s) < sim.workspace_bytes(70, 1)


def test_binomial_checkpointing_against_oracle_and_in_a_graph():
    b = _batch("quad_1024", 4, 150)
    gq0, gqd0, gtau = _grad_parity(b, K=-5)
    # after one call outside capture (schedule upload), the pass can be captured
    sim = _sim(b)
    q0, qd0, tau, ws, qT, qdT, _ = _rollout(sim, b, K=-5)
    gqT, gqdT = 2 * qT, torch.zeros_like(qdT)
    out = sim.backward(tau, b.dt, -5, ws, gqT, gqdT)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cap = sim.backward(tau, b.dt, -5, ws, gqT, gqdT)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        for x, y in zip(out, cap):
            assert torch.equal(x, y)
    assert np.allclose(out[2].cpu().numpy(), gtau, rtol=1e-4, atol=1e-6)
