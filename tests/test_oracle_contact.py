"""Pins of the oracle's contact resolution inside a step (contact.inc:
contact spheres against the ground plane, MLCP of Eq. mlcp on the contact
impulses, projected Gauss-Seidel, velocity update; Sec. 4.1 "Collision
resolution") against what mechanics fixes:

* without contact the step is the plain step, bitwise;
* a ball hitting the ground stops vertically with the impulse m v_n, and
  keeps its tangential and angular velocity when frictionless;
* a sliding point mass loses mu lambda_n / m of tangential speed per step,
  or sticks;
* the contact Jacobian equals central differences of the contact point's
  world position, computed with the independent world-frame Newton-Euler
  kinematics (tests/dyn_ref.py), and A = J M^-1 J^T with M from the same
  reference; a struck pendulum's impulse is -v_n / (J M^-1 J^T);
* Baumgarte stabilisation pushes a penetrating sphere out at beta phi / dt;
* the rollout gradient through persistent contact equals central
  differences of the rollout.  CPU only.
"""
import numpy as np
import pytest

import dyn_ref as R
import oracle as O
from paper_2109_07719_amd import synth

G = 9.81


def _ball(mass=2.0, inertia=0.008):
    return synth.System(parent=np.array([-1], np.int32), jtype=np.array([synth.FREE], np.int32),
                        E_T=np.eye(3)[None], r_T=np.zeros((1, 3)), axis=np.array([[0.0, 0.0, 1.0]]),
                        mass=np.array([mass]), com=np.zeros((1, 3)),
                        Ic=np.array([[inertia, inertia, inertia, 0.0, 0.0, 0.0]]))


def _quat(rng):
    qt = rng.normal(size=4)
    return qt / np.linalg.norm(qt)


def test_without_contact_the_step_is_the_plain_step():
    rng = np.random.default_rng(0)
    for seed in (2000, 2001, 2002):
        s, q0, qd0, tau = synth.tree_system(seed, 1, nmax=10, random_frames=True)
        m = O.Model(s)
        C = O.Contacts(np.arange(s.n), rng.normal(0, 0.1, (s.n, 3)), np.full(s.n, 0.05))
        # lift the whole tree: the root joint sits 100 m up
        s.r_T[0] = [0.0, 100.0, 0.0]
        m = O.Model(s)
        q1, qd1, na, _ = O.step_contact(m, C, q0, qd0, tau[0], 1e-3)
        p1, pd1 = O.step(m, q0, qd0, tau[0], 1e-3)
        assert na == 0 and np.array_equal(q1, p1) and np.array_equal(qd1, pd1)


def test_frictionless_ball_impact_closed_form():
    """Inelastic impact through the centre: lambda_n = m (-v_n) with v_n the
    normal velocity before the impulse, which becomes zero; the tangential
    and angular velocities are unchanged (the impulse acts on the vertical
    through the centre)."""
    rng = np.random.default_rng(1)
    for _ in range(10):
        mass = rng.uniform(0.5, 3.0)
        m = O.Model(_ball(mass))
        C = O.Contacts([0], [[0.0, 0.0, 0.0]], [0.1], mu=0.0, beta=0.0, niter=60)
        qt = _quat(rng)
        q = np.r_[rng.normal(size=3), qt]
        q[1] = 0.1 - rng.uniform(1e-4, 1e-2)
        Rw = R._quat_R(qt)                     # body -> world
        v_world = np.r_[rng.normal(), -rng.uniform(0.5, 3.0), rng.normal()]
        w = rng.normal(size=3)
        qd = np.r_[w, Rw.T @ v_world]
        q1, qd1, na, lam = O.step_contact(m, C, q, qd, [], 1e-3)
        # the velocity before the impulse is the plain step's (pinned on its own)
        _, qdm = O.step(m, q, qd, [], 1e-3)
        vm = Rw @ qdm[3:]
        assert na == 1
        assert abs(lam[0] - mass * (-vm[1])) < 1e-10 * mass * abs(vm[1])
        v1 = Rw @ qd1[3:]
        assert abs(v1[1]) < 1e-12 and np.allclose(v1[[0, 2]], vm[[0, 2]], atol=1e-12)
        assert np.allclose(qd1[:3], qdm[:3], atol=1e-12)
        assert abs(vm[1] - (v_world[1] - G * 1e-3)) < 1e-2      # about v_n - g dt


@pytest.mark.parametrize("vx,vz", [(2.0, 0.001), (-1.5, 0.0), (0.0005, -0.0003)])
def test_sliding_point_mass_friction(vx, vz):
    """A point mass resting on the ground (contact point at the centre of
    mass): the normal impulse cancels gravity over the step, and each
    tangential velocity drops by at most mu lambda_n / m (box friction
    per axis): it slides at that rate or sticks."""
    mass, mu, dt = 1.5, 0.4, 1e-3
    m = O.Model(_ball(mass))
    C = O.Contacts([0], [[0.0, 0.0, 0.0]], [0.0], mu=mu, beta=0.0, niter=60)
    q = np.array([0.0, -1e-4, 0.0, 0.0, 0.0, 0.0, 1.0])
    qd = np.array([0.0, 0.0, 0.0, vx, 0.0, vz])
    q1, qd1, na, lam = O.step_contact(m, C, q, qd, [], dt)
    lam_n = mass * G * dt
    assert na == 1 and abs(lam[0] - lam_n) < 1e-12
    dv = mu * lam_n / mass
    for k, v in ((3, vx), (5, vz)):
        expect = np.sign(v) * max(abs(v) - dv, 0.0)
        assert abs(qd1[k] - expect) < 1e-12, (k, qd1[k], expect)
    assert abs(qd1[4]) < 1e-12


def _tree_with_contacts(seed, rng, prismatic=0.3):
    s, q0, qd0, tau = synth.tree_system(seed, 1, nmax=8, random_frames=True, prismatic=prismatic)
    k = min(s.n, 4)
    links = rng.choice(s.n, size=k, replace=False)
    C = O.Contacts(links, rng.normal(0, 0.2, (k, 3)), rng.uniform(0.02, 0.1, k))
    return s, q0, qd0, tau, C


def _world_point(s, q, link, c_local):
    Rs, o, *_ = R.kinematics(s, q, np.zeros(s.nv), np.zeros(s.nv), np.array([0.0, -G, 0.0]))
    return o[link] + Rs[link] @ c_local


def test_assembly_against_newton_euler_kinematics_and_mass_matrix():
    """J (rows: normal e_y, tangents e_x, e_z of each contact point) equals
    central differences of the point's world position under the independent
    Newton-Euler kinematics, with the point fixed in its link; M^-1 J^T
    equals the solve with that reference's mass matrix; A is symmetric
    positive definite.  Every contact is made active by lowering the ground
    to the lowest sphere (the gap is measured, not assumed)."""
    rng = np.random.default_rng(3)
    checked = 0
    for seed in range(2000, 2012):
        s, q0, qd0, tau, C = _tree_with_contacts(seed, rng)
        q = rng.normal(0, 0.8, s.nq)
        # lift the tree so that every sphere straddles y = 0: move the root
        # frame so that the lowest sphere centre sits just above its radius
        m = O.Model(s)
        ys = [_world_point(s, q, l, c)[1] - r for l, c, r in zip(C.link, C.center, C.radius)]
        s.r_T[0] = s.r_T[0] - np.array([0.0, max(ys) + 1e-3, 0.0])   # all gaps negative
        m = O.Model(s)
        act, phi, J, MJ = O.contact_assembly(m, C, q)
        assert len(act) == C.n
        M = R.mass_matrix(s, q)
        h = 1e-6
        for a, k in enumerate(act):
            l, c, r = C.link[k], C.center[k], C.radius[k]
            Rs, o, *_ = R.kinematics(s, q, np.zeros(s.nv), np.zeros(s.nv), np.array([0.0, -G, 0.0]))
            c_low = c - r * (Rs[l].T @ np.array([0.0, 1.0, 0.0]))      # lowest point, link coordinates
            assert abs((o[l] + Rs[l] @ c)[1] - r - phi[a]) < 1e-12
            Jfd = np.zeros((3, s.nv))
            for j in range(s.nv):
                dq = np.zeros(s.nq)
                dq[j] = h
                Jfd[:, j] = (_world_point(s, q + dq, l, c_low) - _world_point(s, q - dq, l, c_low)) / (2 * h)
            assert np.allclose(J[3 * a:3 * a + 3], Jfd[[1, 0, 2]], atol=1e-8), (seed, a)
        assert np.allclose(MJ, np.linalg.solve(M, J.T), atol=1e-10 * max(1.0, np.abs(MJ).max()))
        A = J @ MJ
        assert np.allclose(A, A.T, atol=1e-10 * np.abs(A).max())
        assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > -1e-12
        checked += 1
    assert checked == 12


def test_struck_pendulum_impulse_is_the_effective_mass_law():
    """A pendulum (revolute about z, tip sphere) swinging into the ground,
    frictionless: one contact, lambda = -v_n / (J M^-1 J^T) with M and J
    from the Newton-Euler reference, and the tip's normal velocity after the
    step is zero."""
    rng = np.random.default_rng(4)
    for _ in range(6):
        Lk = rng.uniform(0.3, 1.0)
        s = synth.System(parent=np.array([-1], np.int32), jtype=np.array([synth.REVOLUTE], np.int32),
                         E_T=np.eye(3)[None], r_T=np.array([[0.0, Lk * 0.5, 0.0]]), axis=np.array([[0.0, 0.0, 1.0]]),
                         mass=np.array([rng.uniform(0.5, 2.0)]), com=np.array([[Lk / 2, 0.0, 0.0]]),
                         Ic=np.array([[0.01, 0.01, 0.02, 0.0, 0.0, 0.0]]))
        C = O.Contacts([0], [[Lk, 0.0, 0.0]], [0.02], mu=0.0, beta=0.0, niter=80)
        m = O.Model(s)
        # angle at which the tip sphere just touches the ground: Lk/2 + Lk sin q - 0.02 = -1e-4
        qc = np.arcsin((-1e-4 + 0.02 - Lk * 0.5) / Lk)
        q, qd = np.array([qc]), np.array([-rng.uniform(0.5, 2.0)])    # swinging down
        q1, qd1, na, lam = O.step_contact(m, C, q, qd, [0.0], 1e-3)
        assert na == 1
        Mref = R.mass_matrix(s, q)
        h = 1e-6
        Rs, o, *_ = R.kinematics(s, q, np.zeros(1), np.zeros(1), np.array([0.0, -G, 0.0]))
        low = np.array([Lk, 0.0, 0.0]) - 0.02 * (Rs[0].T @ np.array([0.0, 1.0, 0.0]))
        Jn = (_world_point(s, q + h, 0, low)[1] - _world_point(s, q - h, 0, low)[1]) / (2 * h)
        qdd = O.fd(m, q, qd, [0.0])
        vn = Jn * (qd[0] + 1e-3 * qdd[0])
        lam_ref = -vn / (Jn * Jn / Mref[0, 0])
        assert abs(lam[0] - lam_ref) < 1e-7 * abs(lam_ref), (lam[0], lam_ref)
        assert abs(Jn * qd1[0]) < 1e-10


def test_baumgarte_pushes_out_at_beta_phi_over_dt():
    """A ball at rest, sunk by phi below the ground, frictionless: with
    Baumgarte factor beta its vertical velocity after the step is
    -beta phi / dt (the normal row's a = v_n + beta phi / dt is zero)."""
    m = O.Model(_ball(1.0))
    for beta, sink in ((0.2, 1e-3), (0.5, 3e-3)):
        C = O.Contacts([0], [[0.0, 0.0, 0.0]], [0.1], mu=0.0, beta=beta, niter=60)
        q = np.array([0.0, 0.1 - sink, 0.0, 0.0, 0.0, 0.0, 1.0])
        q1, qd1, na, lam = O.step_contact(m, C, q, np.zeros(6), [], 1e-3)
        assert na == 1 and abs(qd1[4] - beta * sink / 1e-3) < 1e-10


def _resting_chain(T, mu):
    """A planar 3-link chain (revolute joints about z) lying along x on the
    ground, spheres on the middle of link 1 and the tip of link 2 sunk 2 mm:
    gravity keeps both in contact along the rollout and under small
    perturbations, so the step map is smooth there (no Baumgarte term: its
    push-out velocity would lift the chain off)."""
    s, q0, qd0, tau = synth.chain_system(3, 7, T)
    s.r_T[0] = [0.0, 0.05 - 2e-3, 0.0]
    C = O.Contacts([1, 2], [[0.25, 0.0, 0.0], [0.5, 0.0, 0.0]], [0.05, 0.05], mu=mu, beta=0.0, niter=40)
    rng = np.random.default_rng(5)
    q0 = np.array([0.0, 0.0, 0.0]) + rng.normal(0, 1e-3, 3)
    qd0 = rng.normal(0, 1e-3, 3)
    tau = rng.normal(0, 0.5, (T, 3))
    return s, q0, qd0, tau, C


@pytest.mark.parametrize("mu", [0.0, 0.8])
def test_rollout_gradient_with_contact_central_differences(mu):
    """The gradient through a rollout in persistent contact (the step map's
    exact derivative applied in reverse time) against central differences
    of the rollout, h = 1e-6 (good to about 1e-9 here), on every q0 and qd0
    entry and sampled tau."""
    T, dt = 40, 1e-3
    s, q0, qd0, tau, C = _resting_chain(T, mu)
    m = O.Model(s)
    qT, qdT, nc = O.rollout_contact(m, C, q0, qd0, tau, dt)
    assert nc.min() >= 1
    rng = np.random.default_rng(6)
    wq, wv = rng.normal(size=3), rng.normal(size=3)
    gq0, gqd0, gtau = O.rollout_contact_grad(m, C, q0, qd0, tau, dt, wq, wv)

    def L(a, b_, u):
        x, y, n_ = O.rollout_contact(m, C, a, b_, u, dt)
        assert np.array_equal(n_, nc)      # same contacts: the kink is not crossed
        return wq @ x + wv @ y

    h = 1e-6
    scale = max(np.abs(gq0).max(), np.abs(gqd0).max(), np.abs(gtau).max())
    for j in range(3):
        e = np.eye(3)[j] * h
        assert abs((L(q0 + e, qd0, tau) - L(q0 - e, qd0, tau)) / (2 * h) - gq0[j]) < 1e-8 * scale
        assert abs((L(q0, qd0 + e, tau) - L(q0, qd0 - e, tau)) / (2 * h) - gqd0[j]) < 1e-8 * scale
    for _ in range(6):
        t, j = int(rng.integers(0, T)), int(rng.integers(0, 3))
        up, dn = tau.copy(), tau.copy()
        up[t, j] += h
        dn[t, j] -= h
        assert abs((L(q0, qd0, up) - L(q0, qd0, dn)) / (2 * h) - gtau[t, j]) < 1e-8 * scale


def test_friction_gradient_of_a_sliding_point_mass_closed_form():
    """A point mass sliding along x on the ground (contact at the centre of
    mass, frictional box bound active every step) loses mu g dt of speed per
    step: v_T = v_0 - T mu g dt and x_T = x_0 + dt sum_t v_t, so
    dv_T/dmu = -T g dt and dx_T/dmu = -g dt^2 T (T + 1) / 2."""
    T, dt, mu = 30, 1e-3, 0.4
    m = O.Model(_ball(1.5))
    C = O.Contacts([0], [[0.0, 0.0, 0.0]], [0.0], mu=mu, beta=0.0, niter=40)
    q0 = np.array([0.0, -1e-4, 0.0, 0.0, 0.0, 0.0, 1.0])
    qd0 = np.array([0.0, 0.0, 0.0, 2.0, 0.0, 0.0])
    for k, expect in ((3, -T * G * dt), (0, -G * dt * dt * T * (T + 1) / 2)):
        gq, gv = np.zeros(7), np.zeros(6)
        if k == 3:
            gv[3] = 1.0
        else:
            gq[0] = 1.0
        *_, gmu = O.rollout_contact_grad(m, C, q0, qd0, np.zeros((T, 0)), dt, gq, gv, mu_grad=True)
        assert abs(gmu - expect) < 1e-10 * abs(expect), (k, gmu, expect)


def test_friction_gradient_central_differences():
    """dL/dmu through a landing with friction against central differences
    of the rollout in mu (persistent contact set over the window)."""
    from paper_2109_07719_amd import synth
    s, q0, qd0, tau, links, centers, radii = synth.landing_quadruped(3100, 60, drop=-0.002)
    m = O.Model(s)
    rng = np.random.default_rng(8)
    wq, wv = rng.normal(size=s.nq), rng.normal(size=s.nv)
    mu, h = 0.3, 1e-6

    def L(mu_):
        C_ = O.Contacts(links, centers, radii, mu=mu_, beta=0.2, niter=30)
        x, y, n_ = O.rollout_contact(m, C_, q0, qd0, tau, 1e-3)
        return wq @ x + wv @ y, n_

    C = O.Contacts(links, centers, radii, mu=mu, beta=0.2, niter=30)
    *_, gmu = O.rollout_contact_grad(m, C, q0, qd0, tau, 1e-3, wq, wv, mu_grad=True)
    (lp, n1), (lm, n2) = L(mu + h), L(mu - h)
    assert np.array_equal(n1, n2)
    fd = (lp - lm) / (2 * h)
    print("dL/dmu", gmu, "central differences", fd)
    assert abs(gmu) > 1e-3 and abs(fd - gmu) < 1e-6 * max(1.0, abs(gmu))
