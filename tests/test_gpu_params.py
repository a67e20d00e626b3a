"""GPU parity of the model-parameter gradients against the FP64 oracle:
every link's inertial parameters (mass, first moment, rotational inertia
about the link origin) and every 1-dof link's placement and axis (joint-frame
rotation, joint origin, axis along the unit sphere), summed over the
rollout.  Every kernel variant: general trees with random frames,
free-floating quadrupeds, serial chains with random axes (the library rotates
link frames internally and must turn the gradients back into the caller's
frames), and every adjoint schedule (pipelined K = 1, one-wave K = 1, segment
replay K > 1, store-all K = 0).
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
                 synth.quadruped_system(3001, T), synth.tree_system(2002, T), synth.chain_system(2, 40, T)]
    else:
        import test_gpu_chains as C
        b = C._chains(T, twisted=True, f32=False)
        draws = [(s, b.q0[a:a1], b.qd0[v:v1], np.asarray(b.tau[:, u:u1]))
                 for s, a, a1, v, v1, u, u1 in zip(b.systems, *C._pairs(b))]
    b = synth.make_batch(draws, 1e-3, name=kind)
    return synth.round_to_f32(b) if f32 else b


def _gpu(b, K, dtype, tiling=None):
    from paper_2109_07719_amd.sim import Sim
    sim = Sim(b.systems, b.gravity, dtype=dtype)
    if tiling is not None:
        sim.set_tiling(*tiling)
    q0, qd0, tau = _t(b.q0, dtype), _t(b.qd0, dtype), _t(b.tau, dtype)
    ws = sim.new_workspace(b.T, K)
    qT, qdT, _ = sim.forward(q0, qd0, tau, b.dt, K=K, workspace=ws)
    out = sim.backward(tau, b.dt, K, ws, 2 * qT, qdT, params=True)
    assert sim.status() == 0
    return [x.cpu().numpy() for x in out]


def _oracle(b):
    qo, vo, uo = b.offsets()

    def one(i):
        m = O.Model(b.systems[i], b.gravity)
        q0, qd0 = b.q0[qo[i]:qo[i + 1]], b.qd0[vo[i]:vo[i + 1]]
        tau = np.asarray(b.tau[:, uo[i]:uo[i + 1]], dtype=np.float64)
        qT, qdT = O.rollout(m, q0, qd0, tau, b.dt)
        return O.rollout_grad_params(m, q0, qd0, tau, b.dt, 2 * qT, qdT)[3:5]

    return O.map_threads(one, range(len(b.systems)))


def _compare(b, out, ref, tol, floor):
    off = np.cumsum([0] + [s.n for s in b.systems])
    for k, what in ((3, "inertial"), (4, "placement/axis")):
        errs = [rel(out[k][off[i]:off[i + 1]], ref[i][k - 3], floor) for i in range(len(b.systems))]
        print(b.name, what, "parameter-gradient rel errs", ["%.1e" % e for e in errs])
        assert max(errs) < tol, (what, errs)


@pytest.mark.parametrize("K", [1, 3, 0])
@pytest.mark.parametrize("kind", ["mixed", "chains"])
def test_param_gradients_fp64_round_off(kind, K):
    b = _batch(kind, 150, f32=False)
    _compare(b, _gpu(b, K, torch.float64), _oracle(b), 1e-9, FLOOR_F64)


@pytest.mark.parametrize("kind", ["mixed", "chains"])
def test_param_gradients_fp32(kind):
    b = _batch(kind, 300, f32=True)
    _compare(b, _gpu(b, 1, torch.float32), _oracle(b), TOL_GRAD_F32, 1e-6)


def test_param_gradients_one_wave_fp64():
    b = _batch("mixed", 90, f32=False)
    _compare(b, _gpu(b, 1, torch.float64, (2, 1, 0)), _oracle(b), 1e-9, FLOOR_F64)


def test_param_gradients_one_wave_and_pipelined_agree():
    b = _batch("mixed", 120, f32=True)
    for k in (3, 4):
        a = _gpu(b, 1, torch.float32, (4, 2, 1))[k]
        c = _gpu(b, 1, torch.float32, (1, 1, 0))[k]
        d = _gpu(b, 1, torch.float32, (2, 1, 1))[k]
        assert rel(c, a) < 1e-5
        assert np.array_equal(a, d)


def test_param_gradients_optional():
    """Without the parameter outputs the other gradients are the same up to
    rounding: the two are separate kernel instantiations, and the compiler
    may fuse multiplies and adds differently where the parameter adjoints
    reuse an intermediate."""
    from paper_2109_07719_amd.sim import Sim
    b = _batch("mixed", 60, f32=True)
    sim = Sim(b.systems, b.gravity, dtype=torch.float32)
    q0, qd0, tau = (_t(x, torch.float32) for x in (b.q0, b.qd0, b.tau))
    ws = sim.new_workspace(b.T, 1)
    qT, qdT, _ = sim.forward(q0, qd0, tau, b.dt, K=1, workspace=ws)
    g1 = sim.backward(tau, b.dt, 1, ws, 2 * qT, qdT)
    g2 = sim.backward(tau, b.dt, 1, ws, 2 * qT, qdT, params=True)
    for x, y in zip(g1, g2[:3]):
        assert rel(x.cpu().numpy(), y.cpu().numpy()) < 1e-5
    assert g2[3].shape == (sum(s.n for s in b.systems), 10)
    assert g2[4].shape == (sum(s.n for s in b.systems), 9)
    # a free root has no placement or axis
    off = np.cumsum([0] + [s.n for s in b.systems])
    gf = g2[4].cpu().numpy()
    for i, s in enumerate(b.systems):
        if s.jtype[0] == synth.FREE:
            assert not np.any(gf[off[i]])
