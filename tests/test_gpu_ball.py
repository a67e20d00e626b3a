"""GPU parity for spherical (ball) joints (X_J = rot(R(quat)^T), S = [1; 0],
quaternion state, angular velocity and three torques per joint) against the
FP64 oracle: forward dynamics, rollouts, input gradients under every
adjoint schedule, model-parameter gradients and the tangent rollout.  One
handle mixes trees with ball joints (identity and random joint frames, one
with a ball joint at a fixed root), free-floating quadrupeds on ball hips, a
prismatic tree and all-revolute systems, so the ball variant runs every
joint type at once.  A ball joint's quaternion gradient is the gradient along
the unit sphere: the oracle's is compared with its radial part removed, and
tangent directions are compared along tangents of the sphere.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from helpers import (FLOOR_F64, TOL_GRAD_F32, TOL_QDD_F32, TOL_STATE_F32, ball_tangent, oracle_fd, oracle_grads,
                     rel)
from paper_2109_07719_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _t(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def _batch(T, f32):
    draws = [synth.ball_tree_system(2400 + i, T, random_frames=(i % 2 == 0), spherical=0.3 + 0.1 * i)
             for i in range(5)]
    draws += [synth.ball_quadruped_system(3400 + i, T) for i in range(3)]
    s, q0, qd0, tau = synth.tree_system(2450, T, random_frames=True)
    draws.append(synth.with_spherical_joints(s, q0, qd0, tau, (0, 2), 2451))  # ball joint at a fixed root
    draws += [synth.tree_system(2460, T, random_frames=True, prismatic=0.4), synth.chain_system(7, 1460, T)]
    b = synth.make_batch(draws, 1e-3, name="ball")
    return synth.round_to_f32(b) if f32 else b


def _sim(b, dtype, tiling=None):
    from paper_2109_07719_amd.sim import Sim
    sim = Sim(b.systems, b.gravity, dtype=dtype)
    if tiling is not None:
        sim.set_tiling(*tiling)
    return sim


def _ball_slices(b):
    """(system, q offset) of every ball joint's quaternion in the batch."""
    qo = b.offsets()[0]
    out = []
    for i, s in enumerate(b.systems):
        k = qo[i]
        for j in range(s.n):
            if s.jtype[j] == synth.SPHERICAL:
                out.append((i, k))
            k += 7 if s.jtype[j] == synth.FREE else 4 if s.jtype[j] == synth.SPHERICAL else 1
    return out


def _random_state(b, rng, scale=0.5):
    qo, vo, uo = b.offsets()
    q = rng.normal(0, scale, qo[-1])
    for i, s in enumerate(b.systems):
        if s.jtype[0] == synth.FREE:
            qt = rng.normal(size=4)
            q[qo[i] + 3:qo[i] + 7] = qt / np.linalg.norm(qt)
    for _, k in _ball_slices(b):
        qt = rng.normal(size=4)
        q[k:k + 4] = qt / np.linalg.norm(qt)
    r = lambda x: x.astype(np.float32).astype(np.float64)
    q = r(q)
    # unit to FP64 round-off: off the sphere the free root's Galilean shift
    # no longer leaves a ball joint's dynamics unchanged (an O(|q|^2 - 1)
    # difference from the oracle's unnormalised formula)
    for _, k in _ball_slices(b):
        q[k:k + 4] /= np.linalg.norm(q[k:k + 4])
    return q, r(rng.normal(0, scale, vo[-1])), r(rng.normal(0, 1, uo[-1]))


def test_handle_takes_the_ball_variant():
    b = _batch(1, f32=False)
    info = _sim(b, torch.float64).info
    assert info["has_ball"] == 1 and info["chain"] == 0 and info["has_free"] == 1
    assert info["nq"] == b.q0.size and info["nv"] == b.qd0.size and info["nu"] == b.tau.shape[1]
    assert len(_ball_slices(b)) >= 15


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_aba_qdd(dtype):
    b = _batch(1, f32=False)
    td = torch.float64 if dtype == "f64" else torch.float32
    q, qd, tau = _random_state(b, np.random.default_rng(21), 0.5 if dtype == "f64" else 0.2)
    qdd = _sim(b, td).aba(_t(q, td), _t(qd, td), _t(tau, td)).cpu().numpy()
    ref = oracle_fd(b, q, qd, tau)
    vo = b.offsets()[1]
    floor, tol = (FLOOR_F64, 1e-11) if dtype == "f64" else (1e-6, TOL_QDD_F32)
    errs = [rel(qdd[vo[i]:vo[i + 1]], ref[i], floor) for i in range(len(b.systems))]
    print("ball qdd errs", ["%.1e" % e for e in errs])
    assert max(errs) < tol, errs


def test_state_after_1000_steps_fp32():
    b = _batch(1000, f32=True)
    sim = _sim(b, torch.float32)
    qT, qdT, _ = sim.forward(_t(b.q0, torch.float32), _t(b.qd0, torch.float32), _t(b.tau, torch.float32), b.dt,
                             workspace=None)
    qT, qdT = qT.cpu().numpy(), qdT.cpu().numpy()
    ref = oracle_grads(b, lambda i, q, v: (np.zeros_like(q), np.zeros_like(v)))
    qo, vo, _ = b.offsets()
    errs = [rel(np.r_[qT[qo[i]:qo[i + 1]], qdT[vo[i]:vo[i + 1]]], np.r_[ref[i][3], ref[i][4]])
            for i in range(len(b.systems))]
    print("state after 1000 steps", ["%.1e" % e for e in errs])
    assert max(errs) < TOL_STATE_F32, errs
    # the integrator keeps every ball quaternion on the unit sphere
    for _, k in _ball_slices(b):
        assert abs(np.linalg.norm(qT[k:k + 4]) - 1) < 1e-6
    assert sim.status() == 0


def _gpu_grads(b, K, dtype, tiling=None, params=False):
    sim = _sim(b, dtype, tiling)
    q0, qd0, tau = _t(b.q0, dtype), _t(b.qd0, dtype), _t(b.tau, dtype)
    ws = sim.new_workspace(b.T, K)
    qT, qdT, _ = sim.forward(q0, qd0, tau, b.dt, K=K, workspace=ws)
    out = sim.backward(tau, b.dt, K, ws, 2 * qT, qdT, params=params)
    assert sim.status() == 0
    return [x.cpu().numpy() for x in out]


def _check_grads(b, g, tol, floor):
    ref = oracle_grads(b, lambda i, q, v: (2 * q, v))
    qo, vo, uo = b.offsets()
    worst, elem = {}, 0.0
    for i, s in enumerate(b.systems):
        gq_ref = ball_tangent(s, b.q0[qo[i]:qo[i + 1]], ref[i][0])
        for nm, x, y in (("gq0", g[0][qo[i]:qo[i + 1]], gq_ref), ("gqd0", g[1][vo[i]:vo[i + 1]], ref[i][1]),
                         ("gtau", g[2][:, uo[i]:uo[i + 1]], ref[i][2])):
            worst[nm] = max(worst.get(nm, 0.0), rel(x, y, floor))
            elem = max(elem, float(np.max(np.abs(np.asarray(x) - y), initial=0.0)))
    print({k: "%.2e" % v for k, v in worst.items()}, "elementwise max abs %.2e" % elem)
    assert max(worst.values()) < tol, worst
    # the returned quaternion gradients are tangent to the sphere
    for _, k in _ball_slices(b):
        qh = b.q0[k:k + 4] / np.linalg.norm(b.q0[k:k + 4])
        assert abs(float(g[0][k:k + 4] @ qh)) <= 10 * tol * max(np.linalg.norm(g[0][k:k + 4]), 1.0)


@pytest.mark.parametrize("K,tiling", [(1, (4, 2, 1)), (1, (1, 1, 0)), (3, None), (0, None), (-4, None)])
def test_gradients_fp64_round_off(K, tiling):
    b = _batch(150, f32=False)
    _check_grads(b, _gpu_grads(b, K, torch.float64, tiling), 1e-9, FLOOR_F64)


@pytest.mark.parametrize("K", [1, 0])
def test_gradients_fp32(K):
    b = _batch(300, f32=True)
    _check_grads(b, _gpu_grads(b, K, torch.float32), TOL_GRAD_F32, 1e-6)


def _oracle_params(b):
    qo, vo, uo = b.offsets()

    def one(i):
        m = O.Model(b.systems[i], b.gravity)
        q0, qd0 = b.q0[qo[i]:qo[i + 1]], b.qd0[vo[i]:vo[i + 1]]
        tau = np.asarray(b.tau[:, uo[i]:uo[i + 1]], dtype=np.float64)
        qT, qdT = O.rollout(m, q0, qd0, tau, b.dt)
        return O.rollout_grad_params(m, q0, qd0, tau, b.dt, 2 * qT, qdT)[3:5]

    return O.map_threads(one, range(len(b.systems)))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_param_gradients(dtype):
    f32 = dtype == "f32"
    b = _batch(300 if f32 else 150, f32=f32)
    out = _gpu_grads(b, 1, torch.float32 if f32 else torch.float64, params=True)
    ref = _oracle_params(b)
    off = np.cumsum([0] + [s.n for s in b.systems])
    floor, tol = (1e-6, TOL_GRAD_F32) if f32 else (FLOOR_F64, 1e-9)
    for k in (3, 4):
        errs = [rel(out[k][off[i]:off[i + 1]], ref[i][k - 3], floor) for i in range(len(b.systems))]
        print("parameter-gradient errs", k, ["%.1e" % e for e in errs])
        assert max(errs) < tol, (k, errs)


def test_pipelined_and_one_wave_adjoints_agree_fp32():
    b = _batch(120, f32=True)
    a = _gpu_grads(b, 1, torch.float32, (4, 2, 1), params=True)
    c = _gpu_grads(b, 1, torch.float32, (1, 1, 0), params=True)
    d = _gpu_grads(b, 1, torch.float32, (2, 1, 1), params=True)
    for x, y, z in zip(a, c, d):
        assert rel(y, x) < 1e-5
        assert np.array_equal(x, z)


def test_tangent_rollout_fp64_against_complex_step():
    import test_gpu_jvp as J
    b = _batch(150, f32=False)
    dq0, dqd0, dtau = J._direction(b, 23)
    for _, k in _ball_slices(b):  # directions along the unit sphere
        qh = b.q0[k:k + 4] / np.linalg.norm(b.q0[k:k + 4])
        dq0[k:k + 4] -= (dq0[k:k + 4] @ qh) * qh
    sim = _sim(b, torch.float64)
    f = lambda x: _t(x, torch.float64)
    _, _, dqT, dqdT = (x.cpu().numpy() for x in sim.forward_jvp(f(b.q0), f(b.qd0), f(b.tau), f(dq0), f(dqd0),
                                                                 f(dtau), b.dt))
    J._compare(b, dqT, dqdT, J._oracle_jvp(b, dq0, dqd0, dtau), 1e-9, FLOOR_F64)
    # and the adjoint kernel is its transpose along such directions
    rng = np.random.default_rng(24)
    wq, wqd = rng.normal(size=b.q0.size), rng.normal(size=b.qd0.size)
    ws = sim.new_workspace(b.T, 1)
    sim.forward(f(b.q0), f(b.qd0), f(b.tau), b.dt, K=1, workspace=ws)
    gq0, gqd0, gtau = sim.backward(f(b.tau), b.dt, 1, ws, f(wq), f(wqd))
    lhs = float(wq @ dqT + wqd @ dqdT)
    rhs = float(gq0.cpu().numpy() @ dq0 + gqd0.cpu().numpy() @ dqd0 + np.sum(gtau.cpu().numpy() * dtau))
    assert abs(lhs - rhs) < 1e-10 * max(abs(lhs), abs(rhs), 1.0), (lhs, rhs)
