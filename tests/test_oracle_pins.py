"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test ties the oracle to a closed form, an independent textbook
formalism (world-frame classical Newton-Euler in tests/dyn_ref.py), an
invariant, or a derivative of the pinned forward map.  Together they are
chosen so that a dropped term, a wrong sign or index, or a transposed
operand anywhere in the oracle's ABA, integrator or adjoint fails one of
them.
"""
import itertools
from dataclasses import replace

import numpy as np
import pytest

import dyn_ref as R
import oracle as O
from paper_2109_07719_amd import synth


def _rand_rot(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    return R._quat_R(q)


def _random_tree(parent, rng, random_frames=True, prismatic=False):
    n = len(parent)
    axis = rng.normal(size=(n, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    E_T = np.stack([_rand_rot(rng) if random_frames else np.eye(3) for _ in range(n)])
    Icd = rng.uniform(0.01, 0.1, (n, 3))
    Ic = np.concatenate([Icd, rng.uniform(-0.003, 0.003, (n, 3))], axis=1)
    jtype = (rng.uniform(size=n) < 0.5).astype(np.int32) * synth.PRISMATIC if prismatic else np.zeros(n, np.int32)
    return synth.System(parent=np.asarray(parent, np.int32), jtype=jtype,
                        E_T=E_T, r_T=rng.normal(0, 0.4, (n, 3)), axis=axis,
                        mass=rng.uniform(0.5, 2.0, n), com=rng.uniform(-0.25, 0.25, (n, 3)),
                        Ic=Ic)


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------- forward

def all_parent_arrays(n):
    return itertools.product(*[range(-1, i) for i in range(n)])


def test_aba_equals_dense_solve_every_tree_up_to_4_links():
    """ABA reaches M(q)^-1 (tau - C(q, qd)) exactly (Sec. 3, ABA); M and C
    from an independent world-frame Newton-Euler.  Every parent array with
    parent[i] < i for n <= 4 (33 shapes, forests included), random axes,
    frames, offsets, inertias (with products of inertia) and states."""
    rng = np.random.default_rng(11)
    count = 0
    for n in range(1, 5):
        for parent in all_parent_arrays(n):
            s = _random_tree(parent, rng)
            m = O.Model(s)
            for _ in range(3):
                q, qd, tau = rng.normal(0, 1, n), rng.normal(0, 1, n), rng.normal(0, 1, n)
                assert _rel(O.fd(m, q, qd, tau), R.forward_dynamics(s, q, qd, tau)) < 1e-12
            count += 1
    assert count == 33


@pytest.mark.parametrize("seed", [2000, 2001, 2002])
def test_aba_equals_dense_solve_branched_trees(seed):
    s, q0, qd0, tau = synth.tree_system(seed, 1, random_frames=True)
    m = O.Model(s)
    rng = np.random.default_rng(seed)
    q, qd = rng.normal(0, 1, s.n), rng.normal(0, 1, s.n)
    assert _rel(O.fd(m, q, qd, tau[0]), R.forward_dynamics(s, q, qd, tau[0])) < 1e-11


def test_free_base_dense_solve_and_momentum_balance():
    """Free-floating root (the quadruped's 19/18 dimensions, Sec. 6.1): the
    joint rows of inverse dynamics at the oracle's accelerations equal tau,
    and the six root rows (net wrench of inertial minus gravity forces on
    the whole tree) vanish -- total momentum changes only by gravity."""
    for seed in range(3000, 3004):
        s, q0, qd0, tau = synth.quadruped_system(seed, 1)
        assert (s.nq, s.nv, s.nu) == (19, 18, 12)
        rng = np.random.default_rng(seed)
        qt = rng.normal(size=4)
        q = q0.copy()
        q[3:7] = qt / np.linalg.norm(qt)
        q[7:] = rng.normal(0, 1, 12)
        qd = rng.normal(0, 1, 18)
        m = O.Model(s)
        qdd = O.fd(m, q, qd, tau[0])
        res = R.inverse_dynamics(s, q, qd, qdd)
        scale = np.abs(R.inverse_dynamics(s, q, qd, np.zeros(18))).max()
        assert np.abs(res[:6]).max() < 1e-12 * scale
        assert np.abs(res[6:] - tau[0]).max() < 1e-12 * scale
        assert _rel(qdd, R.forward_dynamics(s, q, qd, tau[0])) < 1e-11


def _pendulum(m_=1.3, c=0.4, Izz=0.05):
    return synth.System(parent=np.array([-1], np.int32), jtype=np.zeros(1, np.int32),
                        E_T=np.eye(3)[None], r_T=np.zeros((1, 3)),
                        axis=np.array([[0.0, 0.0, 1.0]]), mass=np.array([m_]),
                        com=np.array([[c, 0.0, 0.0]]), Ic=np.array([[0.01, 0.02, Izz, 0, 0, 0]]))


def test_single_pendulum_closed_form():
    """(Izz + m c^2) th'' = tau - m g c cos(th), th measured from +x, gravity -y."""
    s = _pendulum()
    m = O.Model(s)
    for th, thd, tau in [(0.0, 0.0, 0.0), (0.3, 0.7, 0.5), (-1.2, -2.0, 1.0), (2.0, 5.0, -3.0)]:
        ref = (tau - 1.3 * 9.81 * 0.4 * np.cos(th)) / (0.05 + 1.3 * 0.4 ** 2)
        assert abs(O.fd(m, [th], [thd], [tau])[0] - ref) < 1e-13 * max(1, abs(ref))


def test_single_pendulum_small_oscillation_period():
    """Hanging at th = -pi/2, small oscillations have period
    2 pi sqrt((Izz + m c^2) / (m g c)); checked to O(dt) + O(amplitude^2)."""
    s = _pendulum()
    m = O.Model(s)
    dt, T = 1e-4, 30000
    q, qd, tr = O.rollout(m, [-np.pi / 2 + 1e-3], [0.0], np.zeros((T, 1)), dt, traj=True)
    th = tr[:, 0] + np.pi / 2
    up = np.where((th[:-1] < 0) & (th[1:] >= 0))[0]
    # linear interpolation of upward zero crossings
    tc = (up + (-th[up]) / (th[up + 1] - th[up])) * dt
    period = np.mean(np.diff(tc))
    ref = 2 * np.pi * np.sqrt((0.05 + 1.3 * 0.16) / (1.3 * 9.81 * 0.4))
    assert abs(period - ref) / ref < 2e-3


def test_double_pendulum_closed_form():
    """Planar 2R arm (link length l1, COMs c1, c2 on the links): textbook
    mass matrix, Coriolis and gravity terms."""
    m1, m2, c1, c2, l1, I1, I2 = 1.1, 0.7, 0.2, 0.3, 0.5, 0.04, 0.03
    s = synth.System(parent=np.array([-1, 0], np.int32), jtype=np.zeros(2, np.int32),
                     E_T=np.stack([np.eye(3)] * 2), r_T=np.array([[0, 0, 0], [l1, 0, 0.0]]),
                     axis=np.array([[0, 0, 1.0], [0, 0, 1.0]]), mass=np.array([m1, m2]),
                     com=np.array([[c1, 0, 0], [c2, 0, 0.0]]),
                     Ic=np.array([[0.01, 0.01, I1, 0, 0, 0], [0.01, 0.01, I2, 0, 0, 0]]))
    m = O.Model(s)
    g = 9.81
    rng = np.random.default_rng(5)
    for _ in range(20):
        q, qd, tau = rng.normal(0, 2, 2), rng.normal(0, 2, 2), rng.normal(0, 2, 2)
        M11 = I1 + I2 + m1 * c1 ** 2 + m2 * (l1 ** 2 + c2 ** 2 + 2 * l1 * c2 * np.cos(q[1]))
        M12 = I2 + m2 * (c2 ** 2 + l1 * c2 * np.cos(q[1]))
        M22 = I2 + m2 * c2 ** 2
        h = m2 * l1 * c2 * np.sin(q[1])
        C = np.array([-h * (2 * qd[0] * qd[1] + qd[1] ** 2), h * qd[0] ** 2])
        G = np.array([(m1 * c1 + m2 * l1) * g * np.cos(q[0]) + m2 * c2 * g * np.cos(q[0] + q[1]),
                      m2 * c2 * g * np.cos(q[0] + q[1])])
        ref = np.linalg.solve(np.array([[M11, M12], [M12, M22]]), tau - C - G)
        assert _rel(O.fd(m, q, qd, tau), ref) < 1e-12


def test_gravity_along_joint_axes_is_inert():
    """With gravity along the z joint axes of a planar chain, gravity does no
    work: the accelerations equal those with zero gravity."""
    s, q0, qd0, tau = synth.chain_system(7, 0, 1)
    a = O.fd(O.Model(s, gravity=(0, 0, -9.81)), q0, qd0, tau[0])
    b = O.fd(O.Model(s, gravity=(0, 0, 0)), q0, qd0, tau[0])
    assert _rel(a, b) < 1e-13


def test_energy_drift_is_first_order_in_dt():
    """Semi-implicit Euler on a passive chain: the largest energy deviation
    over 1 s shrinks linearly with dt (ratio 0.5 +- 0.15 per halving)."""
    s, q0, qd0, _ = synth.chain_system(7, 0, 1)
    m = O.Model(s)
    q0 = q0 + 0.5
    E0 = R.energy(s, q0, qd0)
    drifts = []
    for dt in (1e-3, 5e-4, 2.5e-4):
        T = int(round(1.0 / dt))
        _, _, tr = O.rollout(m, q0, qd0, np.zeros((T, 7)), dt, traj=True)
        idx = np.linspace(0, T - 1, 200).astype(int)
        drifts.append(max(abs(R.energy(s, tr[k, :7], tr[k, 7:]) - E0) for k in idx))
    for a, b in zip(drifts, drifts[1:]):
        assert 0.35 < b / a < 0.65, drifts


def test_semi_implicit_euler_step_and_no_secular_energy_growth():
    """One step is q1 = q + dt (qd + dt qdd), qd1 = qd + dt qdd (the
    semi-implicit scheme), and, being symplectic, it keeps the energy of a
    passive pendulum bounded over 20 s (an explicit Euler step would let it
    grow steadily)."""
    s = _pendulum()
    m = O.Model(s)
    q, qd, tau, dt = np.array([0.4]), np.array([-1.3]), np.array([0.2]), 1e-3
    qdd = O.fd(m, q, qd, tau)
    q1, qd1 = O.step(m, q, qd, tau, dt)
    assert abs(qd1[0] - (qd[0] + dt * qdd[0])) < 1e-15
    assert abs(q1[0] - (q[0] + dt * qd1[0])) < 1e-15
    T = 20000
    _, _, tr = O.rollout(m, [0.3], [0.0], np.zeros((T, 1)), dt, traj=True)
    E = np.array([R.energy(s, tr[k, :1], tr[k, 1:]) for k in range(0, T, 50)])
    dE = np.abs(E - R.energy(s, np.array([0.3]), np.array([0.0])))
    first = dE[: len(dE) // 10].max()
    assert dE[-len(dE) // 10:].max() < 2.0 * first


# ---------------------------------------------------------------- adjoint

def test_single_step_tau_bar_is_Minv_qdd_bar():
    """dqdd/dtau = M^-1, so the reverse ABA must return tau_bar = M^-1 qdd_bar
    (M from the independent Newton-Euler)."""
    rng = np.random.default_rng(3)
    for parent in [(-1, 0, 1, 2, 3, 4, 5), (-1, 0, 0, 1, 1, 2, -1, 6)]:
        s = _random_tree(parent, rng)
        m = O.Model(s)
        q, qd, tau = rng.normal(0, 1, s.n), rng.normal(0, 1, s.n), rng.normal(0, 1, s.n)
        qb = rng.normal(0, 1, s.n)
        _, _, tb = O.fd_vjp(m, q, qd, tau, qb)
        M = R.mass_matrix(s, q)
        assert _rel(tb, np.linalg.solve(M.T, qb)) < 1e-11


def _id_jacobians(s, q, qd, qdd, h=1e-30):
    """d ID / dq and d ID / dqd by complex step on the Newton-Euler reference."""
    n = len(q)
    Jq = np.zeros((len(qdd), n))
    Jv = np.zeros((len(qdd), len(qd)))
    for j in range(n):
        e = np.zeros(n, complex)
        e[j] = 1j * h
        Jq[:, j] = R.inverse_dynamics(s, q + e, qd.astype(complex), qdd.astype(complex)).imag / h
    for j in range(len(qd)):
        e = np.zeros(len(qd), complex)
        e[j] = 1j * h
        Jv[:, j] = R.inverse_dynamics(s, q.astype(complex), qd + e, qdd.astype(complex)).imag / h
    return Jq, Jv


def test_single_step_state_adjoint_matches_inverse_dynamics_jacobian():
    """Implicit differentiation of ID(q, qd, FD(q, qd, tau)) = tau gives
    q_bar = -(dID/dq)^T tau_bar and qd_bar = -(dID/dqd)^T tau_bar.  The
    reverse ABA reaches the same numbers by a different route."""
    rng = np.random.default_rng(4)
    for parent in [(-1, 0, 1, 2, 3), (-1, 0, 0, 1, 2, 2)]:
        s = _random_tree(parent, rng)
        m = O.Model(s)
        q, qd, tau = rng.normal(0, 1, s.n), rng.normal(0, 1, s.n), rng.normal(0, 1, s.n)
        qb = rng.normal(0, 1, s.n)
        gq, gqd, tb = O.fd_vjp(m, q, qd, tau, qb)
        qdd = O.fd(m, q, qd, tau)
        Jq, Jv = _id_jacobians(s, q, qd, qdd)
        assert _rel(gq, -Jq.T @ tb) < 1e-10
        assert _rel(gqd, -Jv.T @ tb) < 1e-10


def test_free_base_single_step_adjoint_matches_inverse_dynamics_jacobian():
    """Same identity with a free root, on the base velocity, the base
    position and the joint angles (the quaternion has a scale gauge and is
    checked through complex-step rollouts instead)."""
    s, q0, qd0, tau = synth.quadruped_system(3007, 1)
    rng = np.random.default_rng(8)
    q = q0.copy()
    qt = rng.normal(size=4)
    q[3:7] = qt / np.linalg.norm(qt)
    q[7:] = rng.normal(0, 0.5, 12)
    qd = rng.normal(0, 1, 18)
    m = O.Model(s)
    qb = rng.normal(0, 1, 18)
    gq, gqd, tb = O.fd_vjp(m, q, qd, tau[0], qb)
    qdd = O.fd(m, q, qd, tau[0])
    Jq, Jv = _id_jacobians(s, q, qd, qdd)
    M = R.mass_matrix(s, q)
    fb = np.linalg.solve(M.T, qb)       # adjoint of the full generalised force
    assert _rel(tb, fb[6:]) < 1e-10
    assert _rel(gqd, -Jv.T @ fb) < 1e-10
    sel = np.r_[0:3, 7:19]
    assert _rel(gq[sel], (-Jq.T @ fb)[sel]) < 1e-10


def _loss_seed(m, qT):
    return 2 * qT, np.zeros(m.nv)


def test_rollout_gradient_complex_step_chain():
    """Whole-rollout gradient of L = sum q_T^2 by the adjoint method (Eq.
    adj_r) against complex-step derivatives of the (pinned) forward rollout,
    on every q0, qd0 entry and a sample of tau entries."""
    b = synth.workload("chain7_fp64", T=200)
    s = b.systems[0]
    m = O.Model(s)
    qT, _ = O.rollout(m, b.q0, b.qd0, b.tau, b.dt)
    gq0, gqd0, gtau, _, _ = O.rollout_grad(m, b.q0, b.qd0, b.tau, b.dt, *_loss_seed(m, qT))
    h = 1e-30

    def L(q0, qd0, tau):
        qT, _ = O.rollout_complex(m, q0, qd0, tau, b.dt)
        return np.sum(qT ** 2)

    for j in range(7):
        e = np.zeros(7, complex)
        e[j] = 1j * h
        assert abs(L(b.q0 + e, b.qd0.astype(complex), b.tau.astype(complex)).imag / h - gq0[j]) \
            < 1e-10 * max(1, abs(gq0[j]))
        assert abs(L(b.q0.astype(complex), b.qd0 + e, b.tau.astype(complex)).imag / h - gqd0[j]) \
            < 1e-10 * max(1, abs(gqd0[j]))
    rng = np.random.default_rng(0)
    scale = np.abs(gtau).max()
    for _ in range(12):
        t, j = int(rng.integers(0, 200)), int(rng.integers(0, 7))
        tc = b.tau.astype(complex)
        tc[t, j] += 1j * h
        assert abs(L(b.q0.astype(complex), b.qd0.astype(complex), tc).imag / h - gtau[t, j]) \
            < 1e-10 * scale


def test_rollout_vjp_dot_product_tree_and_traj_seed():
    """<VJP(w), v> = <w, JVP(v)> for the whole rollout of a branched tree,
    with a dense seed on every intermediate state (traj) and on x^T; the JVP
    is the complex-step directional derivative of the forward rollout."""
    s, q0, qd0, tau = synth.tree_system(2005, 60, random_frames=True)
    m = O.Model(s)
    rng = np.random.default_rng(1)
    T, nx = tau.shape[0], s.nq + s.nv
    gtraj = rng.normal(size=(T, nx))
    gqT, gqdT = rng.normal(size=s.nq), rng.normal(size=s.nv)
    gq0, gqd0, gtau, _, _ = O.rollout_grad(m, q0, qd0, tau, 5e-4, gqT, gqdT, gtraj)
    v0, vd0, vt = rng.normal(size=s.nq), rng.normal(size=s.nv), rng.normal(size=tau.shape)
    h = 1e-30
    # JVP of traj and x^T via complex-step rollouts with traj recorded step by step
    q, qd = q0 + 1j * h * v0, qd0 + 1j * h * vd0
    dot = 0.0
    for t in range(T):
        # one complex step at a time
        q, qd = O.rollout_complex(m, q, qd, (tau[t] + 1j * h * vt[t])[None, :], 5e-4)
        dot += gtraj[t] @ np.concatenate([q.imag, qd.imag]) / h
    dot += gqT @ q.imag / h + gqdT @ qd.imag / h
    lhs = gq0 @ v0 + gqd0 @ vd0 + np.sum(gtau * vt)
    assert abs(lhs - dot) < 1e-10 * max(abs(dot), 1.0)


def test_free_base_rollout_gradient_complex_step():
    """Quadruped rollout (quaternion integration and normalisation on the
    path): adjoint gradient against complex-step derivatives for every
    entry of q0 (quaternion included: both sides differentiate the same
    homogeneous rotation formula) and qd0, plus sampled tau entries."""
    s, q0, qd0, tau = synth.quadruped_system(3001, 150)
    m = O.Model(s)
    rng = np.random.default_rng(2)
    wq, wv = rng.normal(size=19), rng.normal(size=18)

    def Lr(qT, qdT):
        return wq @ qT + wv @ qdT

    gq0, gqd0, gtau, qT, qdT = O.rollout_grad(m, q0, qd0, tau, 1e-3, wq, wv)
    h = 1e-30

    def Lc(a, b_, t):
        qT, qdT = O.rollout_complex(m, a, b_, t, 1e-3)
        return Lr(qT, qdT)

    scale = max(np.abs(gq0).max(), np.abs(gqd0).max())
    for j in range(19):
        e = np.zeros(19, complex)
        e[j] = 1j * h
        d = Lc(q0 + e, qd0.astype(complex), tau.astype(complex)).imag / h
        assert abs(d - gq0[j]) < 1e-9 * scale, j
    for j in range(18):
        e = np.zeros(18, complex)
        e[j] = 1j * h
        d = Lc(q0.astype(complex), qd0 + e, tau.astype(complex)).imag / h
        assert abs(d - gqd0[j]) < 1e-9 * scale, j
    for _ in range(8):
        t, j = int(rng.integers(0, 150)), int(rng.integers(0, 12))
        tc = tau.astype(complex)
        tc[t, j] += 1j * h
        d = Lc(q0.astype(complex), qd0.astype(complex), tc).imag / h
        assert abs(d - gtau[t, j]) < 1e-9 * np.abs(gtau).max()


def test_rollout_gradient_central_differences_tree():
    """Central differences (h = 1e-6) on a branched tree with random frames."""
    s, q0, qd0, tau = synth.tree_system(2003, 100, random_frames=True)
    m = O.Model(s)
    dt = 5e-4

    def L(a, b_, t):
        qT, qdT = O.rollout(m, a, b_, t, dt)
        return np.sum(qT ** 2) + 0.5 * np.sum(qdT ** 2)

    qT, qdT = O.rollout(m, q0, qd0, tau, dt)
    gq0, gqd0, gtau, _, _ = O.rollout_grad(m, q0, qd0, tau, dt, 2 * qT, qdT)
    h = 1e-6
    for j in range(0, s.n, 3):
        e = np.zeros(s.n)
        e[j] = h
        assert abs((L(q0 + e, qd0, tau) - L(q0 - e, qd0, tau)) / (2 * h) - gq0[j]) < 1e-6 * max(1, abs(gq0[j]))
        assert abs((L(q0, qd0 + e, tau) - L(q0, qd0 - e, tau)) / (2 * h) - gqd0[j]) < 1e-6 * max(1, abs(gqd0[j]))


@pytest.mark.parametrize("which", ["chain", "quad"])
def test_checkpoint_interval_changes_no_arithmetic(which):
    """Storing every step, every K steps with segment replay, or every
    intermediate (store-all) must give bitwise-identical gradients: the
    recompute repeats the same arithmetic (Sec. 4.2; App. B)."""
    if which == "chain":
        s, q0, qd0, tau = synth.chain_system(7, 1000, 237)
    else:
        s, q0, qd0, tau = synth.quadruped_system(3000, 237)
    m = O.Model(s)
    rng = np.random.default_rng(9)
    gqT, gqdT = rng.normal(size=s.nq), rng.normal(size=s.nv)
    gtraj = rng.normal(size=(237, s.nq + s.nv))
    ref = O.rollout_grad(m, q0, qd0, tau, 1e-3, gqT, gqdT, gtraj, K=1)
    for K in (0, 2, 10, 100, 237, 500):
        got = O.rollout_grad(m, q0, qd0, tau, 1e-3, gqT, gqdT, gtraj, K=K)
        for a, b_ in zip(ref, got):
            assert np.array_equal(a, b_), K


def test_rollout_final_state_matches_stepwise():
    s, q0, qd0, tau = synth.quadruped_system(3002, 20)
    m = O.Model(s)
    q, qd = q0, qd0
    for t in range(20):
        q, qd = O.step(m, q, qd, tau[t], 1e-3)
    qT, qdT = O.rollout(m, q0, qd0, tau, 1e-3)
    assert np.array_equal(q, qT) and np.array_equal(qd, qdT)
    assert abs(np.linalg.norm(qT[3:7]) - 1) < 1e-14


def test_adjoint_along_own_trajectory_equals_checkpointed_adjoint():
    """Feeding the oracle's own per-step states to the reverse sweep as
    checkpoints reproduces its checkpointed adjoint bitwise."""
    s, q0, qd0, tau = synth.quadruped_system(3004, 150)
    m = O.Model(s)
    qT, qdT, tr = O.rollout(m, q0, qd0, tau, 1e-3, traj=True)
    states = np.concatenate([np.r_[q0, qd0][None], tr[:-1]])
    rng = np.random.default_rng(0)
    gqT, gqdT, gtr = rng.normal(size=19), rng.normal(size=18), rng.normal(size=tr.shape)
    a = O.adjoint_along(m, states, tau, 1e-3, gqT, gqdT, gtr)
    b = O.rollout_grad(m, q0, qd0, tau, 1e-3, gqT, gqdT, gtr)
    assert all(np.array_equal(x, y) for x, y in zip(a, b[:3]))


# ------------------------------------------------------- inertial-parameter gradients

def _inertial_params(s):
    """Per link (m, h = m c, I_O = I_c - m [c]x^2 as xx yy zz xy xz yz)."""
    th = np.zeros((s.n, 10))
    for i in range(s.n):
        m, c = float(s.mass[i]), np.asarray(s.com[i], dtype=float)
        Ic = np.asarray(s.Ic[i], dtype=float)
        J = np.array([[Ic[0], Ic[3], Ic[4]], [Ic[3], Ic[1], Ic[5]], [Ic[4], Ic[5], Ic[2]]])
        IO = J + m * (np.dot(c, c) * np.eye(3) - np.outer(c, c))
        th[i] = [m, *(m * c), IO[0, 0], IO[1, 1], IO[2, 2], IO[0, 1], IO[0, 2], IO[1, 2]]
    return th


def _with_inertial_params(s, th):
    """The same system with the links' inertial parameters replaced."""
    mass, com, Ic = np.zeros(s.n), np.zeros((s.n, 3)), np.zeros((s.n, 6))
    for i in range(s.n):
        m, h = th[i, 0], th[i, 1:4]
        IO = np.array([[th[i, 4], th[i, 7], th[i, 8]], [th[i, 7], th[i, 5], th[i, 9]], [th[i, 8], th[i, 9], th[i, 6]]])
        J = IO - (np.dot(h, h) * np.eye(3) - np.outer(h, h)) / m
        mass[i], com[i] = m, h / m
        Ic[i] = [J[0, 0], J[1, 1], J[2, 2], J[0, 1], J[0, 2], J[1, 2]]
    return synth.System(parent=s.parent, jtype=s.jtype, E_T=s.E_T, r_T=s.r_T, axis=s.axis, mass=mass, com=com,
                        Ic=Ic)


def _param_problems():
    tree = synth.tree_system(2005, 120, random_frames=True)
    quad = synth.quadruped_system(3007, 120)
    chain = synth.chain_system(5, 11, 120)
    return [("tree", tree, 5e-4), ("quad", quad, 1e-3), ("chain", chain, 1e-3)]


def _param_loss(s, q0, qd0, tau, dt):
    m = O.Model(s)
    qT, qdT = O.rollout(m, q0, qd0, tau, dt)
    return float(np.sum(qT ** 2) + 0.5 * np.sum(qdT ** 2)), qT, qdT


@pytest.mark.parametrize("k", [0, 1, 2])
def test_inertial_parameter_gradient_central_differences(k):
    """Gradient of L = |q_T|^2 + |qd_T|^2 / 2 with respect to every inertial
    parameter of a few links against central differences of the (pinned)
    forward rollout, on a branched tree with random frames, a free-floating
    quadruped and a chain (Sec. 4.1, after Eq. adj_r)."""
    name, (s, q0, qd0, tau), dt = _param_problems()[k]
    _, qT, qdT = _param_loss(s, q0, qd0, tau, dt)
    g = O.rollout_grad_params(O.Model(s), q0, qd0, tau, dt, 2 * qT, qdT)[3]
    th = _inertial_params(s)
    rng = np.random.default_rng(k)
    links = sorted(set([0, s.n - 1] + list(rng.choice(s.n, size=min(3, s.n), replace=False))))
    for i in links:
        for j in range(10):
            if name == "chain" and j not in (0, 1, 2, 6):
                continue   # planar chain: the other parameters do not enter (checked below)
            h = 1e-6 * max(1.0, abs(th[i, j]))
            tp, tm = th.copy(), th.copy()
            tp[i, j] += h
            tm[i, j] -= h
            fd = (_param_loss(_with_inertial_params(s, tp), q0, qd0, tau, dt)[0] -
                  _param_loss(_with_inertial_params(s, tm), q0, qd0, tau, dt)[0]) / (2 * h)
            assert abs(fd - g[i, j]) < 2e-6 * max(1.0, abs(g[i, j]), np.abs(g).max()), (name, i, j, fd, g[i, j])
    if name == "chain":
        # z-axis joints, in-plane gravity: out-of-plane parameters are inert
        assert np.abs(g[:, [3, 4, 5, 7, 8, 9]]).max() < 1e-12 * np.abs(g).max()


@pytest.mark.parametrize("k", [0, 1, 2])
def test_inertial_parameter_gradient_scaling_identity(k):
    """Scaling every inertial parameter and every torque by the same factor
    leaves the motion unchanged (M, C and gravity terms are linear in the
    inertial parameters), so <theta, dL/dtheta> + <tau, dL/dtau> = 0 exactly."""
    name, (s, q0, qd0, tau), dt = _param_problems()[k]
    _, qT, qdT = _param_loss(s, q0, qd0, tau, dt)
    _, _, gtau, g, _, _, _ = O.rollout_grad_params(O.Model(s), q0, qd0, tau, dt, 2 * qT, qdT)
    th = _inertial_params(s)
    a, b = float(np.sum(th * g)), float(np.sum(tau * gtau))
    assert abs(a + b) < 1e-9 * max(abs(a), abs(b)), (a, b)
    assert abs(a) > 1e-6


def test_inertial_parameter_gradient_checkpointing_and_along():
    """K and store-all give bitwise-identical parameter gradients, and the
    sweep along the oracle's own trajectory reproduces them."""
    s, q0, qd0, tau = synth.quadruped_system(3008, 90)
    m = O.Model(s)
    qT, qdT = O.rollout(m, q0, qd0, tau, 1e-3)
    ref = O.rollout_grad_params(m, q0, qd0, tau, 1e-3, 2 * qT, qdT, K=1)[3]
    for K in (0, 7, 90):
        assert np.array_equal(O.rollout_grad_params(m, q0, qd0, tau, 1e-3, 2 * qT, qdT, K=K)[3], ref)
    _, _, traj = O.rollout(m, q0, qd0, tau, 1e-3, traj=True)
    states = np.concatenate([np.r_[q0, qd0][None], traj[:-1]])
    along = O.adjoint_along_params(m, states, tau, 1e-3, 2 * qT, qdT)[3]
    assert np.array_equal(along, ref)



# ------------------------------------------------------------- prismatic joints

def test_aba_equals_dense_solve_every_tree_with_prismatic_joints():
    """As the revolute pin, with every joint of every tree of up to 4 links
    revolute or prismatic at random (X_J = translation by q a, S = [0; a])."""
    rng = np.random.default_rng(12)
    n_prism = 0
    for n in range(1, 5):
        for parent in all_parent_arrays(n):
            for _ in range(2):
                s = _random_tree(parent, rng, prismatic=True)
                n_prism += int(np.sum(s.jtype == synth.PRISMATIC))
                m = O.Model(s)
                q, qd, tau = rng.normal(0, 1, n), rng.normal(0, 1, n), rng.normal(0, 1, n)
                assert _rel(O.fd(m, q, qd, tau), R.forward_dynamics(s, q, qd, tau)) < 1e-12
    assert n_prism > 40


def test_cartpole_closed_form():
    """Cart (prismatic along x) and pole (revolute about z, COM at distance l):
    M = [[mc + mp, -mp l s], [-mp l s, Ip + mp l^2]], bias
    [-mp l c thd^2, mp g l c] with s, c = sin, cos of the pole angle."""
    s, _, _, _ = synth.cartpole_system(5, 1)
    m = O.Model(s)
    mc, mp, l, Ip, g = s.mass[0], s.mass[1], s.com[1][0], s.Ic[1][2], 9.81
    rng = np.random.default_rng(1)
    for _ in range(20):
        q, qd, tau = rng.normal(0, 1.5, 2), rng.normal(0, 2, 2), rng.normal(0, 1, 2)
        sn, cs = np.sin(q[1]), np.cos(q[1])
        M = np.array([[mc + mp, -mp * l * sn], [-mp * l * sn, Ip + mp * l * l]])
        h = np.array([-mp * l * cs * qd[1] ** 2, mp * g * l * cs])
        assert _rel(O.fd(m, q, qd, tau), np.linalg.solve(M, tau - h)) < 1e-12


def test_rollout_gradient_complex_step_with_prismatic_joints():
    """Adjoint rollout gradient (prismatic dX/dq = -crm(S) X with S = [0; a])
    against complex-step derivatives, on a tree with random frames and
    prismatic joints, and on the cart-pole; parameter gradients against
    central differences."""
    for s, q0, qd0, tau, dt in (synth.tree_system(2011, 80, nmax=14, random_frames=True, prismatic=0.4) + (5e-4,),
                                synth.cartpole_system(6, 150) + (1e-3,)):
        assert np.any(s.jtype == synth.PRISMATIC)
        m = O.Model(s)
        qT, qdT = O.rollout(m, q0, qd0, tau, dt)
        gq0, gqd0, gtau, gp, _, _, _ = O.rollout_grad_params(m, q0, qd0, tau, dt, 2 * qT, qdT)
        h = 1e-30

        def L(a, b_, t):
            cq, cqd = O.rollout_complex(m, a, b_, t, dt)
            return np.sum(cq ** 2) + 0.5 * np.sum(cqd ** 2)

        for j in range(s.n):
            e = np.zeros(s.n, complex)
            e[j] = 1j * h
            assert abs(L(q0 + e, qd0.astype(complex), tau.astype(complex)).imag / h - gq0[j]) < 1e-9 * max(1, abs(gq0[j]))
            assert abs(L(q0.astype(complex), qd0 + e, tau.astype(complex)).imag / h - gqd0[j]) < 1e-9 * max(1, abs(gqd0[j]))
        t0 = np.zeros_like(tau, dtype=complex)
        t0[len(tau) // 2, s.n - 1] = 1j * h
        assert abs(L(q0.astype(complex), qd0.astype(complex), tau + t0).imag / h - gtau[len(tau) // 2, s.n - 1]) \
            < 1e-9 * max(1, np.abs(gtau).max())
        th = _inertial_params(s)
        for i in (0, s.n - 1):
            for j in (0, 1, 4, 7):
                hh = 1e-6 * max(1.0, abs(th[i, j]))
                tp, tm = th.copy(), th.copy()
                tp[i, j] += hh
                tm[i, j] -= hh
                fd = (_param_loss(_with_inertial_params(s, tp), q0, qd0, tau, dt)[0] -
                      _param_loss(_with_inertial_params(s, tm), q0, qd0, tau, dt)[0]) / (2 * hh)
                assert abs(fd - gp[i, j]) < 2e-6 * max(1.0, np.abs(gp).max())


# ------------------------------------------------------------- placement and axis gradients

def _rodrigues(w):
    """exp([w]x) for a rotation vector w."""
    th = float(np.linalg.norm(w))
    if th < 1e-300:
        return np.eye(3)
    k = w / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * (K @ K)


def _with_frame(s, i, which, d):
    """The same system with link i's joint frame rotated (E_T -> exp(-[d]x) E_T),
    its joint origin moved (r_T + d) or its axis rotated (exp([d]x) a)."""
    E, r, a = s.E_T.copy(), s.r_T.copy(), s.axis.copy()
    if which == "phi":
        E[i] = _rodrigues(-np.asarray(d)) @ E[i]
    elif which == "r":
        r[i] = r[i] + d
    else:
        a[i] = _rodrigues(np.asarray(d)) @ a[i]
    return synth.System(parent=s.parent, jtype=s.jtype, E_T=E, r_T=r, axis=a, mass=s.mass, com=s.com, Ic=s.Ic)


def _frame_problems():
    tree = synth.tree_system(2012, 100, nmax=16, random_frames=True, prismatic=0.4)
    quad = synth.telescoping_quadruped_system(3009, 100)
    chain = synth.chain_system(5, 12, 100)
    return [("tree", tree, 5e-4), ("quad", quad, 1e-3), ("chain", chain, 1e-3)]


@pytest.mark.parametrize("k", [0, 1, 2])
def test_frame_and_axis_gradients_central_differences(k):
    """Gradients with respect to each 1-dof link's joint-frame rotation, joint
    origin and joint axis against central differences of the (pinned) forward
    rollout: a branched tree with random frames and prismatic joints, a
    free-floating quadruped with sliding knees, a chain.  The axis output is
    the gradient along the unit sphere, so a rotation w of the axis changes
    the loss by (a x axis_bar) . w (Sec. 4.1, after Eq. adj_r)."""
    name, (s, q0, qd0, tau), dt = _frame_problems()[k]
    _, qT, qdT = _param_loss(s, q0, qd0, tau, dt)
    gf = O.rollout_grad_params(O.Model(s), q0, qd0, tau, dt, 2 * qT, qdT)[4]
    scale = np.abs(gf).max()
    assert scale > 1e-3
    rng = np.random.default_rng(20 + k)
    links = [i for i in range(s.n) if s.jtype[i] != synth.FREE]
    links = sorted(set([links[0], links[-1]] + list(rng.choice(links, size=min(3, len(links)), replace=False))))
    h = 1e-6
    for i in links:
        a = s.axis[i] / np.linalg.norm(s.axis[i])
        for which, off in (("phi", 0), ("r", 3), ("w", 6)):
            for j in range(3):
                d = np.zeros(3)
                d[j] = h
                fd = (_param_loss(_with_frame(s, i, which, d), q0, qd0, tau, dt)[0] -
                      _param_loss(_with_frame(s, i, which, -d), q0, qd0, tau, dt)[0]) / (2 * h)
                if which == "w":
                    ref = np.cross(a, gf[i, 6:9])[j]
                else:
                    ref = gf[i, off + j]
                assert abs(fd - ref) < 2e-6 * max(1.0, scale), (name, i, which, j, fd, ref)
        # the axis gradient is tangent to the unit sphere
        assert abs(np.dot(gf[i, 6:9], a)) < 1e-12 * max(1.0, scale)
    # a free root has no placement or axis
    for i in range(s.n):
        if s.jtype[i] == synth.FREE:
            assert not np.any(gf[i])


def test_frame_gradient_invariances_of_a_fixed_base_tree():
    """Moving a fixed-base system's only root joint (all links with it) leaves
    the joint-space motion unchanged, and so does turning it about the
    gravity direction: r_T_bar of the root is zero and phi_bar of the root
    is orthogonal to E_T g.  Exact, not within a difference quotient."""
    for s, q0, qd0, tau, dt in (synth.tree_system(2013, 100, nmax=16, random_frames=True, prismatic=0.3) + (5e-4,),
                                synth.chain_system(6, 13, 100) + (1e-3,)):
        assert np.sum(s.parent < 0) == 1
        m = O.Model(s)
        qT, qdT = O.rollout(m, q0, qd0, tau, dt)
        gf = O.rollout_grad_params(m, q0, qd0, tau, dt, 2 * qT, qdT)[4]
        scale = np.abs(gf).max()
        assert scale > 1e-3
        assert np.abs(gf[0, 3:6]).max() < 1e-10 * scale
        gdir = np.asarray(synth.GRAVITY) / np.linalg.norm(synth.GRAVITY)
        assert abs(np.dot(gf[0, 0:3], s.E_T[0] @ gdir)) < 1e-10 * scale
        # and the other two rotation directions do matter
        assert np.abs(gf[0, 0:3]).max() > 1e-6 * scale


def test_frame_gradients_checkpointing_and_along():
    """K and store-all give bitwise-identical placement and axis gradients,
    and the sweep along the oracle's own trajectory reproduces them."""
    s, q0, qd0, tau = synth.telescoping_quadruped_system(3010, 60)
    m = O.Model(s)
    qT, qdT = O.rollout(m, q0, qd0, tau, 1e-3)
    ref = O.rollout_grad_params(m, q0, qd0, tau, 1e-3, 2 * qT, qdT, K=1)[4]
    for K in (0, 7, 60):
        assert np.array_equal(O.rollout_grad_params(m, q0, qd0, tau, 1e-3, 2 * qT, qdT, K=K)[4], ref)
    _, _, traj = O.rollout(m, q0, qd0, tau, 1e-3, traj=True)
    states = np.concatenate([np.r_[q0, qd0][None], traj[:-1]])
    assert np.array_equal(O.adjoint_along_params(m, states, tau, 1e-3, 2 * qT, qdT)[4], ref)


# ------------------------------------------------------------- joint limits

def test_joint_limit_torque_is_added_to_the_control():
    """By definition the limit acts as an extra joint torque: forward dynamics
    with limits equals forward dynamics without them under tau + tau_limit,
    with tau_limit = -k (q - hi) - d qd above hi, -k (q - lo) - d qd below
    lo and 0 inside, on a tree with random frames and prismatic joints and a
    free-floating quadruped."""
    rng = np.random.default_rng(30)
    for draw in (synth.tree_system(2016, 1, nmax=12, random_frames=True, prismatic=0.4),
                 synth.quadruped_system(3012, 1)):
        s, q0, qd0, _ = synth.with_joint_limits(draw, 31)
        free = s.jtype == synth.FREE
        plain = synth.System(parent=s.parent, jtype=s.jtype, E_T=s.E_T, r_T=s.r_T, axis=s.axis, mass=s.mass,
                             com=s.com, Ic=s.Ic)
        ml, mp = O.Model(s), O.Model(plain)
        qo = np.cumsum([0] + [7 if f else 1 for f in free])
        vo = np.cumsum([0] + [6 if f else 1 for f in free])
        for _ in range(10):
            q = q0 + rng.normal(0, 0.4, q0.size)
            if free[0]:
                q[3:7] = [0, 0, 0, 1]
            qd, tau = rng.normal(0, 1, s.nv), rng.normal(0, 1, s.nu)
            tl = np.zeros(s.nu)
            u = 0
            active = 0
            for i in range(s.n):
                if free[i]:
                    continue
                lo, hi, k, d = s.limits[i]
                qq, vv = q[qo[i]], qd[vo[i]]
                if qq > hi:
                    tl[u] = -k * (qq - hi) - d * vv
                elif qq < lo:
                    tl[u] = -k * (qq - lo) - d * vv
                active += qq > hi or qq < lo
                u += 1
            assert active > 0
            assert _rel(O.fd(ml, q, qd, tau), O.fd(mp, q, qd, tau + tl)) < 1e-13


def test_rollout_gradient_with_joint_limits_complex_step():
    """The adjoint of the limit torque (q_bar += -k u_bar, qd_bar += -d u_bar
    where a limit is active) against complex-step derivatives of rollouts
    that run into the limits, on a chain and a tree with prismatic joints."""
    for draw, dt in ((synth.chain_system(5, 14, 300), 1e-3),
                     (synth.tree_system(2017, 200, nmax=10, random_frames=True, prismatic=0.3), 1e-3)):
        s, q0, qd0, tau = synth.with_joint_limits(draw, 32)
        m = O.Model(s)
        _, _, traj = O.rollout(m, q0, qd0, tau, dt, traj=True)
        lo, hi = s.limits[:, 0], s.limits[:, 1]
        hits = np.sum((traj[:, :s.n] > hi) | (traj[:, :s.n] < lo))
        assert hits > 20, hits
        qT, qdT = O.rollout(m, q0, qd0, tau, dt)
        gq0, gqd0, gtau, _, _ = O.rollout_grad(m, q0, qd0, tau, dt, 2 * qT, qdT)
        h = 1e-30

        def L(a, b_, t):
            cq, cqd = O.rollout_complex(m, a, b_, t, dt)
            return np.sum(cq ** 2) + 0.5 * np.sum(cqd ** 2)

        for j in range(s.n):
            e = np.zeros(s.n, complex)
            e[j] = 1j * h
            assert abs(L(q0 + e, qd0.astype(complex), tau.astype(complex)).imag / h - gq0[j]) < 1e-9 * max(1, abs(gq0[j]))
            assert abs(L(q0.astype(complex), qd0 + e, tau.astype(complex)).imag / h - gqd0[j]) < 1e-9 * max(1, abs(gqd0[j]))
        for t in (0, len(tau) // 3, len(tau) - 1):
            t0 = np.zeros_like(tau, dtype=complex)
            t0[t, s.n // 2] = 1j * h
            ref = L(q0.astype(complex), qd0.astype(complex), tau + t0).imag / h
            assert abs(ref - gtau[t, s.n // 2]) < 1e-9 * max(1, np.abs(gtau).max())


def test_joint_limits_inside_the_range_change_nothing():
    s, q0, qd0, tau = synth.with_joint_limits(synth.chain_system(4, 15, 30), 33, half_range=(50.0, 60.0))
    plain = synth.System(parent=s.parent, jtype=s.jtype, E_T=s.E_T, r_T=s.r_T, axis=s.axis, mass=s.mass,
                         com=s.com, Ic=s.Ic)
    a = O.rollout(O.Model(s), q0, qd0, tau, 1e-3)
    b = O.rollout(O.Model(plain), q0, qd0, tau, 1e-3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ------------------------------------------------------------- spherical joints

def _random_quat(rng):
    qt = rng.normal(size=4)
    return qt / np.linalg.norm(qt)


def _random_state(s, rng, scale=1.0):
    """q (unit quaternions for ball joints and a free root), qd, tau."""
    q = []
    for i in range(s.n):
        if s.jtype[i] == synth.FREE:
            q += list(rng.normal(size=3)) + list(_random_quat(rng))
        elif s.jtype[i] == synth.SPHERICAL:
            q += list(_random_quat(rng))
        else:
            q.append(rng.normal(0, scale))
    return np.array(q), rng.normal(0, scale, s.nv), rng.normal(0, 1, s.nu)


def test_aba_equals_dense_solve_every_tree_with_spherical_joints():
    """ABA with ball joints (S = [1; 0], a 3x3 joint-space inertia per joint)
    reaches M^-1 (tau - C) of the independent world-frame Newton-Euler on
    every parent array of up to 4 links, each joint spherical, prismatic or
    revolute at random, with random frames, offsets and inertias."""
    rng = np.random.default_rng(31)
    count = nsph = 0
    for n in range(1, 5):
        for parent in all_parent_arrays(n):
            u = rng.uniform(size=n)
            jt = np.where(u < 0.5, synth.SPHERICAL, np.where(u < 0.7, synth.PRISMATIC, synth.REVOLUTE))
            s = replace(_random_tree(parent, rng), jtype=jt.astype(np.int32))
            m = O.Model(s)
            for _ in range(3):
                q, qd, tau = _random_state(s, rng)
                assert _rel(O.fd(m, q, qd, tau), R.forward_dynamics(s, q, qd, tau)) < 1e-12
            count += 1
            nsph += int(np.sum(jt == synth.SPHERICAL))
    assert count == 33 and nsph > 30


def test_ball_joint_quadruped_dense_solve_and_momentum_balance():
    """Free-floating base over ball-joint hips: inverse dynamics at the
    oracle's accelerations returns tau on the joints and a zero net wrench
    on the base."""
    for seed in range(3000, 3003):
        s, _, _, tau = synth.ball_quadruped_system(seed, 1)
        assert (s.nq, s.nv, s.nu) == (31, 26, 20)
        q, qd, _ = _random_state(s, np.random.default_rng(seed))
        qdd = O.fd(O.Model(s), q, qd, tau[0])
        res = R.inverse_dynamics(s, q, qd, qdd)
        scale = np.abs(R.inverse_dynamics(s, q, qd, np.zeros(26))).max()
        assert np.abs(res[:6]).max() < 1e-12 * scale
        assert np.abs(res[6:] - tau[0]).max() < 1e-12 * scale


def test_single_body_on_a_ball_joint_obeys_eulers_equations():
    """A rigid body on a ball joint fixed in space turns by Euler's equations
    about the pivot, in body coordinates:
    I_O wdot + w x (I_O w) = tau + c x (m g_b), with I_O = I_c + m (|c|^2 1 -
    c c^T) and g_b the gravity vector in body coordinates (the body-to-world
    rotation is E_T^T R(quat))."""
    rng = np.random.default_rng(41)
    for _ in range(10):
        s = replace(_random_tree((-1,), rng), jtype=np.array([synth.SPHERICAL], np.int32))
        q, w, tau = _random_state(s, rng)
        m_, c = float(s.mass[0]), np.asarray(s.com[0])
        xx, yy, zz, xy, xz, yz = s.Ic[0]
        IO = np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]]) + m_ * (c @ c * np.eye(3) - np.outer(c, c))
        gb = (s.E_T[0].T @ R._quat_R(q)).T @ np.asarray(synth.GRAVITY)
        ref = np.linalg.solve(IO, tau + np.cross(c, m_ * gb) - np.cross(w, IO @ w))
        assert _rel(O.fd(O.Model(s), q, w, tau), ref) < 1e-13


def _ball_problems():
    quad = synth.ball_quadruped_system(3001, 80)
    tree = synth.ball_tree_system(2005, 60, nmax=14, random_frames=True, prismatic=0.2, spherical=0.4)
    return [("quad", quad, 1e-3), ("tree", tree, 5e-4)]


@pytest.mark.parametrize("k", [0, 1])
def test_rollout_gradient_complex_step_with_spherical_joints(k):
    """Rollouts through ball joints (quaternion integration and normalisation
    at every ball joint, a free root on the quadruped): the adjoint gradient
    of a random linear loss against complex-step derivatives of every q0
    entry (quaternions included) and qd0 entry, and of sampled tau entries."""
    name, (s, q0, qd0, tau), dt = _ball_problems()[k]
    assert np.sum(s.jtype == synth.SPHERICAL) >= 2
    m = O.Model(s)
    rng = np.random.default_rng(5 + k)
    wq, wv = rng.normal(size=s.nq), rng.normal(size=s.nv)
    gq0, gqd0, gtau, _, _ = O.rollout_grad(m, q0, qd0, tau, dt, wq, wv)
    h = 1e-30

    def Lc(a, b_, t):
        qT, qdT = O.rollout_complex(m, a, b_, t, dt)
        return wq @ qT + wv @ qdT

    scale = max(np.abs(gq0).max(), np.abs(gqd0).max())
    for j in range(s.nq):
        d = Lc(q0 + 1j * h * np.eye(s.nq)[j], qd0.astype(complex), tau.astype(complex)).imag / h
        assert abs(d - gq0[j]) < 1e-11 * scale, (name, j)
    for j in range(s.nv):
        d = Lc(q0.astype(complex), qd0 + 1j * h * np.eye(s.nv)[j], tau.astype(complex)).imag / h
        assert abs(d - gqd0[j]) < 1e-11 * scale, (name, j)
    for _ in range(10):
        t, j = int(rng.integers(0, tau.shape[0])), int(rng.integers(0, s.nu))
        tc = tau.astype(complex)
        tc[t, j] += 1j * h
        d = Lc(q0.astype(complex), qd0.astype(complex), tc).imag / h
        assert abs(d - gtau[t, j]) < 1e-11 * np.abs(gtau).max(), (name, t, j)


def _qmul(a, b):
    """Hamilton product of quaternions stored (x, y, z, w) (complex-safe)."""
    av, aw, bv, bw = a[:3], a[3], b[:3], b[3]
    return np.r_[aw * bv + bw * av + np.cross(av, bv), aw * bw - av @ bv]


def test_ball_tangent_gradient_is_the_derivative_along_the_sphere():
    """oracle.ball_tangent (the form of a ball joint's quaternion gradient the
    kernels return): orthogonal to each quaternion, and its pairing with the
    velocity of a curve on the unit sphere, q(t) = q (x) (sin(t/2) d, cos(t/2)),
    equals the complex-step derivative of the loss along that curve."""
    name, (s, q0, qd0, tau), dt = _ball_problems()[0]
    m = O.Model(s)
    rng = np.random.default_rng(17)
    wq, wv = rng.normal(size=s.nq), rng.normal(size=s.nv)
    g = O.rollout_grad(m, q0, qd0, tau[:30], dt, wq, wv)[0]
    gt = O.ball_tangent(s, q0, g)
    balls, qi = [], 0
    for i in range(s.n):
        if s.jtype[i] == synth.SPHERICAL:
            balls.append(qi)
        qi += 7 if s.jtype[i] == synth.FREE else 4 if s.jtype[i] == synth.SPHERICAL else 1
    assert len(balls) == 4
    h = 1e-30
    for k in balls:
        q = q0[k:k + 4]
        assert abs(gt[k:k + 4] @ q) < 1e-14 * np.linalg.norm(g[k:k + 4])
        assert abs(g[k:k + 4] @ q) > 1e-3 * np.linalg.norm(g[k:k + 4])  # the full gradient has a radial part
        for _ in range(3):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            th = 1j * h
            qc = q0.astype(complex)
            qc[k:k + 4] = _qmul(q, np.r_[np.sin(th / 2) * d, np.cos(th / 2)])
            qT, qdT = O.rollout_complex(m, qc, qd0.astype(complex), tau[:30].astype(complex), dt)
            deriv = (wq @ qT + wv @ qdT).imag / h
            vel = _qmul(q, np.r_[0.5 * d, 0.0])
            assert abs(gt[k:k + 4] @ vel - deriv) < 1e-11 * max(1.0, abs(deriv)), (k, deriv)


def test_ball_joint_parameter_and_placement_gradients_central_differences():
    """Inertial-parameter and joint-placement gradients of ball-joint links
    against central differences of the forward rollout; a ball joint has no
    axis, so its three axis entries are zero."""
    s, q0, qd0, tau = synth.ball_tree_system(2014, 80, nmax=12, random_frames=True, prismatic=0.2, spherical=0.5)
    dt = 5e-4
    _, qT, qdT = _param_loss(s, q0, qd0, tau, dt)
    out = O.rollout_grad_params(O.Model(s), q0, qd0, tau, dt, 2 * qT, qdT)
    g, gf = out[3], out[4]
    sph = [i for i in range(s.n) if s.jtype[i] == synth.SPHERICAL]
    assert len(sph) >= 2
    th = _inertial_params(s)
    scale = max(np.abs(gf).max(), np.abs(g).max())
    for i in sph[:3]:
        assert not np.any(gf[i, 6:9])
        for which, off in (("phi", 0), ("r", 3)):
            for j in range(3):
                d = np.zeros(3)
                d[j] = 1e-6
                fd = (_param_loss(_with_frame(s, i, which, d), q0, qd0, tau, dt)[0] -
                      _param_loss(_with_frame(s, i, which, -d), q0, qd0, tau, dt)[0]) / 2e-6
                assert abs(fd - gf[i, off + j]) < 2e-6 * max(1.0, scale), (i, which, j, fd, gf[i, off + j])
        for j in range(10):
            hh = 1e-6 * max(1.0, abs(th[i, j]))
            tp, tm = th.copy(), th.copy()
            tp[i, j] += hh
            tm[i, j] -= hh
            fd = (_param_loss(_with_inertial_params(s, tp), q0, qd0, tau, dt)[0] -
                  _param_loss(_with_inertial_params(s, tm), q0, qd0, tau, dt)[0]) / (2 * hh)
            assert abs(fd - g[i, j]) < 2e-6 * max(1.0, scale), (i, j, fd, g[i, j])


def test_ball_joint_integrator_keeps_unit_quaternions_and_first_order_energy_drift():
    """Every ball joint's quaternion stays of unit length after every step,
    and on a passive tree the largest energy deviation over 0.5 s shrinks
    linearly with dt (semi-implicit Euler is first order)."""
    s, q0, qd0, _ = synth.ball_tree_system(2016, 1, nmax=8, spherical=0.6)
    assert np.sum(s.jtype == synth.SPHERICAL) >= 2
    m = O.Model(s)
    qd0 = 3 * qd0
    E0 = R.energy(s, q0, qd0)
    qoff = np.cumsum([0] + [4 if j == synth.SPHERICAL else 1 for j in s.jtype])
    drifts = []
    for dt in (1e-3, 5e-4, 2.5e-4):
        T = int(round(0.5 / dt))
        _, _, tr = O.rollout(m, q0, qd0, np.zeros((T, s.nu)), dt, traj=True)
        for i in np.nonzero(s.jtype == synth.SPHERICAL)[0]:
            nrm = np.linalg.norm(tr[:, qoff[i]:qoff[i] + 4], axis=1)
            assert np.abs(nrm - 1).max() < 1e-14
        idx = np.linspace(0, T - 1, 100).astype(int)
        drifts.append(max(abs(R.energy(s, tr[k, :s.nq], tr[k, s.nq:]) - E0) for k in idx))
    for a, b in zip(drifts, drifts[1:]):
        assert 0.35 < b / a < 0.65, drifts


def test_ball_joint_checkpointing_changes_no_arithmetic():
    """Checkpoint interval and store-all give bitwise-identical gradients
    (inputs, inertial parameters and placements) on the ball-joint
    quadruped, and the sweep along the oracle's own trajectory reproduces
    them."""
    s, q0, qd0, tau = synth.ball_quadruped_system(3011, 50)
    m = O.Model(s)
    qT, qdT = O.rollout(m, q0, qd0, tau, 1e-3)
    ref = O.rollout_grad_params(m, q0, qd0, tau, 1e-3, 2 * qT, qdT, K=1)
    for K in (0, 7, 50):
        out = O.rollout_grad_params(m, q0, qd0, tau, 1e-3, 2 * qT, qdT, K=K)
        for a, b in zip(out[:5], ref[:5]):
            assert np.array_equal(a, b)
    _, _, traj = O.rollout(m, q0, qd0, tau, 1e-3, traj=True)
    states = np.concatenate([np.r_[q0, qd0][None], traj[:-1]])
    along = O.adjoint_along_params(m, states, tau, 1e-3, 2 * qT, qdT)
    for a, b in zip(along[:5], ref[:5]):
        assert np.array_equal(a, b)
