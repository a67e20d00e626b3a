"""GPU parity of the forward-mode (tangent) rollout: the directional
derivative of the final state along a random input direction against the
oracle's complex-step derivative of its (pinned) rollout, which is an
independent forward-mode evaluation; and, on the GPU alone, the
dot-product identity <w, JVP(v)> = <VJP(w), v> between the tangent kernel and
the adjoint kernel.  Every kernel variant: general trees with random frames,
free-floating quadrupeds, serial chains with random axes.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from helpers import FLOOR_F64, TOL_GRAD_F32, rel
from paper_2109_07719_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _t(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def _batch(kind, T, f32):
    if kind == "mixed":
        draws = [synth.chain_system(7, 1000, T), synth.tree_system(2001, T, random_frames=True),
                 synth.quadruped_system(3001, T), synth.tree_system(2002, T)]
    else:
        import test_gpu_chains as C
        b = C._chains(T, twisted=True, f32=False)
        draws = [(s, b.q0[a:a1], b.qd0[v:v1], np.asarray(b.tau[:, u:u1]))
                 for s, a, a1, v, v1, u, u1 in zip(b.systems, *C._pairs(b))]
    b = synth.make_batch(draws, 1e-3, name=kind)
    return synth.round_to_f32(b) if f32 else b


def _direction(b, seed):
    rng = np.random.default_rng(seed)
    qo, vo, uo = b.offsets()
    r = lambda x: x.astype(np.float32).astype(np.float64)
    return r(rng.normal(size=qo[-1])), r(rng.normal(size=vo[-1])), r(rng.normal(size=b.tau.shape))


def _sim(b, dtype):
    from paper_2109_07719_amd.sim import Sim
    return Sim(b.systems, b.gravity, dtype=dtype)


def _oracle_jvp(b, dq0, dqd0, dtau):
    """Complex-step derivative of the oracle rollout along the direction."""
    qo, vo, uo = b.offsets()
    h = 1e-30

    def one(i):
        m = O.Model(b.systems[i], b.gravity)
        q0 = b.q0[qo[i]:qo[i + 1]] + 1j * h * dq0[qo[i]:qo[i + 1]]
        qd0 = b.qd0[vo[i]:vo[i + 1]] + 1j * h * dqd0[vo[i]:vo[i + 1]]
        tau = np.asarray(b.tau[:, uo[i]:uo[i + 1]], dtype=np.float64) + 1j * h * dtau[:, uo[i]:uo[i + 1]]
        qT, qdT = O.rollout_complex(m, q0, qd0, tau, b.dt)
        return qT.imag / h, qdT.imag / h

    return O.map_threads(one, range(len(b.systems)))


def _compare(b, dqT, dqdT, ref, tol, floor):
    qo, vo, _ = b.offsets()
    errs = [rel(np.r_[dqT[qo[i]:qo[i + 1]], dqdT[vo[i]:vo[i + 1]]], np.r_[ref[i][0], ref[i][1]], floor)
            for i in range(len(b.systems))]
    print(b.name, "tangent rel errs", ["%.1e" % e for e in errs])
    assert max(errs) < tol, errs


@pytest.mark.parametrize("T", [1, 150])
@pytest.mark.parametrize("kind", ["mixed", "chains"])
def test_tangent_rollout_fp64_against_complex_step(kind, T):
    b = _batch(kind, T, f32=False)
    dq0, dqd0, dtau = _direction(b, 3)
    sim = _sim(b, torch.float64)
    f = lambda x: _t(x, torch.float64)
    qT, qdT, dqT, dqdT = (x.cpu().numpy() for x in sim.forward_jvp(f(b.q0), f(b.qd0), f(b.tau), f(dq0), f(dqd0),
                                                                    f(dtau), b.dt))
    _compare(b, dqT, dqdT, _oracle_jvp(b, dq0, dqd0, dtau), 1e-9, FLOOR_F64)
    # the value part is the plain rollout
    pq, pqd, _ = sim.forward(f(b.q0), f(b.qd0), f(b.tau), b.dt, workspace=None)
    assert rel(qT, pq.cpu().numpy(), FLOOR_F64) < 1e-13 and rel(qdT, pqd.cpu().numpy(), FLOOR_F64) < 1e-13
    assert sim.status() == 0


@pytest.mark.parametrize("kind", ["mixed", "chains"])
def test_tangent_rollout_fp32(kind):
    b = _batch(kind, 300, f32=True)
    dq0, dqd0, dtau = _direction(b, 4)
    sim = _sim(b, torch.float32)
    f = lambda x: _t(x, torch.float32)
    out = [x.cpu().numpy() for x in sim.forward_jvp(f(b.q0), f(b.qd0), f(b.tau), f(dq0), f(dqd0), f(dtau), b.dt)]
    _compare(b, out[2], out[3], _oracle_jvp(b, dq0, dqd0, dtau), TOL_GRAD_F32, 1e-6)


@pytest.mark.parametrize("kind", ["mixed", "chains"])
def test_tangent_and_adjoint_kernels_are_transposes(kind):
    """<w, J v> = <J^T w, v> for the whole rollout, tangent kernel against
    adjoint kernel (FP64)."""
    b = _batch(kind, 120, f32=False)
    dq0, dqd0, dtau = _direction(b, 5)
    rng = np.random.default_rng(6)
    wq, wqd = rng.normal(size=b.q0.size), rng.normal(size=b.qd0.size)
    sim = _sim(b, torch.float64)
    f = lambda x: _t(x, torch.float64)
    _, _, dqT, dqdT = sim.forward_jvp(f(b.q0), f(b.qd0), f(b.tau), f(dq0), f(dqd0), f(dtau), b.dt)
    ws = sim.new_workspace(b.T, 1)
    sim.forward(f(b.q0), f(b.qd0), f(b.tau), b.dt, K=1, workspace=ws)
    gq0, gqd0, gtau = sim.backward(f(b.tau), b.dt, 1, ws, f(wq), f(wqd))
    lhs = float(wq @ dqT.cpu().numpy() + wqd @ dqdT.cpu().numpy())
    rhs = float(gq0.cpu().numpy() @ dq0 + gqd0.cpu().numpy() @ dqd0 + np.sum(gtau.cpu().numpy() * dtau))
    assert abs(lhs - rhs) < 1e-10 * max(abs(lhs), abs(rhs), 1.0), (lhs, rhs)


def test_tangent_trajectory_output():
    b = _batch("mixed", 40, f32=True)
    dq0, dqd0, dtau = _direction(b, 7)
    sim = _sim(b, torch.float32)
    f = lambda x: _t(x, torch.float32)
    qT, qdT, dqT, dqdT, tr, dtr = sim.forward_jvp(f(b.q0), f(b.qd0), f(b.tau), f(dq0), f(dqd0), f(dtau), b.dt,
                                                  traj=True)
    nq = sim.nq
    assert torch.equal(dtr[-1, :nq], dqT) and torch.equal(dtr[-1, nq:], dqdT) and torch.equal(tr[-1, :nq], qT)
    # row 9 is the tangent after 10 steps
    _, _, dq10, dqd10 = sim.forward_jvp(f(b.q0), f(b.qd0), f(b.tau[:10]), f(dq0), f(dqd0), f(dtau[:10]), b.dt)
    assert torch.equal(dtr[9, :nq], dq10) and torch.equal(dtr[9, nq:], dqd10)
