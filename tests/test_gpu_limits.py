"""GPU parity for joint limits (a one-sided spring and damper outside
[lo, hi] added to the joint control) against the FP64 oracle: forward
dynamics, rollouts that run into the limits, input gradients under every
adjoint schedule, parameter gradients and the tangent rollout.  One handle
mixes limited chains, limited trees with random frames and prismatic joints,
limited free-floating quadrupeds and systems without limits.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from helpers import FLOOR_F64, TOL_GRAD_F32, oracle_fd, oracle_grads, rel
from paper_2109_07719_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _t(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def _batch(T, f32):
    draws = [synth.with_joint_limits(synth.chain_system(7, 1300 + i, T), 40 + i) for i in range(4)]
    draws += [synth.with_joint_limits(synth.tree_system(2300 + i, T, random_frames=True, prismatic=0.3), 50 + i)
              for i in range(4)]
    draws += [synth.with_joint_limits(synth.quadruped_system(3300 + i, T), 60 + i) for i in range(2)]
    draws += [synth.chain_system(5, 1310, T), synth.tree_system(2310, T)]
    b = synth.make_batch(draws, 1e-3, name="limits")
    return synth.round_to_f32(b) if f32 else b


def _sim(b, dtype, tiling=None):
    from paper_2109_07719_amd.sim import Sim
    sim = Sim(b.systems, b.gravity, dtype=dtype)
    if tiling is not None:
        sim.set_tiling(*tiling)
    return sim


def test_rollouts_reach_the_limits():
    b = _batch(300, f32=False)
    hits = 0
    qo, vo, uo = b.offsets()
    for i, s in enumerate(b.systems):
        if s.limits is None:
            continue
        m = O.Model(s, b.gravity)
        _, _, tr = O.rollout(m, b.q0[qo[i]:qo[i + 1]], b.qd0[vo[i]:vo[i + 1]], b.tau[:, uo[i]:uo[i + 1]], b.dt,
                             traj=True)
        qi = 0
        for k in range(s.n):
            if s.jtype[k] == synth.FREE:
                qi += 7
                continue
            hits += int(np.sum((tr[:, qi] > s.limits[k, 1]) | (tr[:, qi] < s.limits[k, 0])))
            qi += 1
    assert hits > 1000, hits


def test_aba_qdd_fp64():
    b = _batch(1, f32=False)
    rng = np.random.default_rng(5)
    qo, vo, uo = b.offsets()
    q = b.q0 + rng.normal(0, 0.4, b.q0.size)
    for i, s in enumerate(b.systems):
        if s.jtype[0] == synth.FREE:
            q[qo[i] + 3:qo[i] + 7] = [0, 0, 0, 1]
    qd, tau = rng.normal(0, 1, vo[-1]), rng.normal(0, 1, uo[-1])
    qdd = _sim(b, torch.float64).aba(_t(q, torch.float64), _t(qd, torch.float64), _t(tau, torch.float64))
    qdd = qdd.cpu().numpy()
    ref = oracle_fd(b, q, qd, tau)
    errs = [rel(qdd[vo[i]:vo[i + 1]], ref[i], FLOOR_F64) for i in range(len(b.systems))]
    assert max(errs) < 1e-11, errs


def _gpu(b, K, dtype, tiling=None, params=False):
    sim = _sim(b, dtype, tiling)
    q0, qd0, tau = _t(b.q0, dtype), _t(b.qd0, dtype), _t(b.tau, dtype)
    ws = sim.new_workspace(b.T, K)
    qT, qdT, _ = sim.forward(q0, qd0, tau, b.dt, K=K, workspace=ws)
    out = sim.backward(tau, b.dt, K, ws, 2 * qT, qdT, params=params)
    assert sim.status() == 0
    return [qT.cpu().numpy(), qdT.cpu().numpy()] + [x.cpu().numpy() for x in out]


def _check(b, g, tol, floor):
    ref = oracle_grads(b, lambda i, q, v: (2 * q, v))
    qo, vo, uo = b.offsets()
    worst = {}
    for i in range(len(b.systems)):
        for nm, x, y in (("qT", g[0][qo[i]:qo[i + 1]], ref[i][3]), ("gq0", g[2][qo[i]:qo[i + 1]], ref[i][0]),
                         ("gqd0", g[3][vo[i]:vo[i + 1]], ref[i][1]), ("gtau", g[4][:, uo[i]:uo[i + 1]], ref[i][2])):
            worst[nm] = max(worst.get(nm, 0.0), rel(x, y, floor))
    print({k: "%.1e" % v for k, v in worst.items()})
    assert max(worst.values()) < tol, worst


@pytest.mark.parametrize("K,tiling", [(1, (4, 2, 1)), (1, (1, 1, 0)), (3, None), (0, None), (-3, None)])
def test_gradients_fp64_round_off(K, tiling):
    b = _batch(200, f32=False)
    _check(b, _gpu(b, K, torch.float64, tiling), 1e-9, FLOOR_F64)


def test_gradients_fp32():
    b = _batch(300, f32=True)
    _check(b, _gpu(b, 1, torch.float32), TOL_GRAD_F32, 1e-6)


def test_param_gradients_fp64():
    b = _batch(150, f32=False)
    out = _gpu(b, 1, torch.float64, params=True)
    qo, vo, uo = b.offsets()

    def one(i):
        m = O.Model(b.systems[i], b.gravity)
        q0, qd0 = b.q0[qo[i]:qo[i + 1]], b.qd0[vo[i]:vo[i + 1]]
        tau = np.asarray(b.tau[:, uo[i]:uo[i + 1]], dtype=np.float64)
        qT, qdT = O.rollout(m, q0, qd0, tau, b.dt)
        return O.rollout_grad_params(m, q0, qd0, tau, b.dt, 2 * qT, qdT)[3:5]

    ref = O.map_threads(one, range(len(b.systems)))
    off = np.cumsum([0] + [s.n for s in b.systems])
    for k in (5, 6):
        errs = [rel(out[k][off[i]:off[i + 1]], ref[i][k - 5], FLOOR_F64) for i in range(len(b.systems))]
        assert max(errs) < 1e-9, (k, errs)


def test_tangent_rollout_fp64_against_complex_step():
    import test_gpu_jvp as J
    b = _batch(150, f32=False)
    dq0, dqd0, dtau = J._direction(b, 23)
    sim = _sim(b, torch.float64)
    f = lambda x: _t(x, torch.float64)
    _, _, dqT, dqdT = (x.cpu().numpy() for x in sim.forward_jvp(f(b.q0), f(b.qd0), f(b.tau), f(dq0), f(dqd0),
                                                                 f(dtau), b.dt))
    J._compare(b, dqT, dqdT, J._oracle_jvp(b, dq0, dqd0, dtau), 1e-9, FLOOR_F64)
