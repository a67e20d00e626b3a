"""The GPU contact step's statements (csrc/contact_step.h, built for the
host) against the FP64 oracle's step with contact, on the CPU: whole
rollouts element by element (FP64 to round-off, FP32 within a stated bar)
and the rollout gradient (each step's Jacobian in dual numbers against the
oracle's complex-step Jacobians, both applied in reverse time)."""
import ctypes

import numpy as np
import pytest

import contact_cases as CC
import dyn_ref as R
import oracle as O
from helpers import contact_emu, rel
from paper_2109_07719_amd import synth
from paper_2109_07719_amd.contact import pack_params

G = (0.0, -9.81, 0.0)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _world_point(s, q, link, c):
    Rs, o, *_ = R.kinematics(s, q, np.zeros(s.nv), np.zeros(s.nv), np.array(G))
    return o[link] + Rs[link] @ c


def _emu_args(s, links, centers, radii, mu, beta, niter):
    par = np.ascontiguousarray(s.parent, np.int32)
    jt = np.ascontiguousarray(s.jtype, np.int32)
    cl = np.ascontiguousarray(links, np.int32)
    g = np.array(G)
    P = np.ascontiguousarray(pack_params(s, centers, radii))
    lim = getattr(s, "limits", None)
    lim = None if lim is None else np.ascontiguousarray(np.asarray(lim, np.float64).reshape(-1))
    keep = (par, jt, cl, g, P, lim)
    return keep, [s.n, _p(par), _p(jt), len(links), _p(cl), mu, beta, niter, _p(g), _p(P)], \
        (_p(lim) if lim is not None else None)


def emu_rollout(s, links, centers, radii, mu, beta, niter, q0, qd0, tau, dt, fp64=True, staged=False):
    keep, a, lim = _emu_args(s, links, centers, radii, mu, beta, niter)
    T = tau.shape[0]
    nx = s.nq + s.nv
    q0, qd0, tau = (np.ascontiguousarray(v, np.float64) for v in (q0, qd0, tau))
    tr = np.zeros((T + 1, nx))
    nc = np.zeros(T, np.int32)
    contact_emu().emu_contact_rollout(int(fp64), *a, _p(q0), _p(qd0), _p(tau), dt, T, _p(tr), _p(nc), lim,
                                      int(staged))
    return tr, nc


def emu_grad(s, links, centers, radii, mu, beta, niter, tr, tau, dt, gqT, gqdT, fp64=True, adjoint=False,
             staged=True):
    """adjoint=False: each step's Jacobian in dual numbers applied in
    reverse time; adjoint=True: the step's reverse statements."""
    keep, a, lim = _emu_args(s, links, centers, radii, mu, beta, niter)
    T = tau.shape[0]
    tau, gqT, gqdT = (np.ascontiguousarray(v, np.float64) for v in (tau, gqT, gqdT))
    gq0, gqd0, gtau, gmu = np.zeros(s.nq), np.zeros(s.nv), np.zeros((T, s.nu)), np.zeros(1)
    args = (int(fp64), *a, _p(np.ascontiguousarray(tr)), _p(tau), dt, T, _p(gqT), _p(gqdT), _p(gq0), _p(gqd0),
            _p(gtau), _p(gmu), lim)
    if adjoint:
        contact_emu().emu_contact_grad_adj(*args, int(staged))
    else:
        contact_emu().emu_contact_grad(*args)
    return gq0, gqd0, gtau, gmu


def _scenes():
    out = []
    s, q0, qd0, tau, links, centers, radii = CC.landing_quadruped(3100, 80)
    out.append(("quadruped landing", s, q0, qd0, tau, links, centers, radii, 0.8, 0.2))
    for seed in (2000, 2003):
        s, q0, qd0, tau, links, centers, radii = CC.grounded_tree(seed, 40)
        s = CC.lower_to_ground(s, q0, links, centers, radii, _world_point, 3e-3)
        out.append((f"tree {seed}", s, q0, qd0, tau, links, centers, radii, 0.5, 0.1))
    s, q0, qd0, tau, links, centers, radii = CC.resting_chain(40)
    out.append(("planar chain", s, q0, qd0, tau, links, centers, radii, 0.8, 0.0))
    # the landing with joint limits around the start pose that the legs run into
    s, q0, qd0, tau, links, centers, radii = CC.landing_quadruped(3100, 80)
    s = synth.with_joint_limits((s, q0, qd0, tau), 77, half_range=(0.002, 0.02))[0]
    out.append(("quadruped landing, joint limits", s, q0, qd0, tau, links, centers, radii, 0.8, 0.2))
    return out


SCENES = _scenes()


@pytest.mark.parametrize("k", range(len(SCENES)), ids=[sc[0] for sc in SCENES])
def test_rollout_fp64_matches_the_oracle(k):
    name, s, q0, qd0, tau, links, centers, radii, mu, beta = SCENES[k]
    dt, niter = 1e-3, 30
    m = O.Model(s, G)
    C = O.Contacts(links, centers, radii, mu=mu, beta=beta, niter=niter)
    _, _, nc_o, tr_o = O.rollout_contact(m, C, q0, qd0, tau, dt, traj=True)
    tr, nc = emu_rollout(s, links, centers, radii, mu, beta, niter, q0, qd0, tau, dt)
    assert np.array_equal(nc, nc_o)
    assert nc.max() >= 1, "the scene must make contact"
    if getattr(s, "limits", None) is not None:
        # the scene must run into its joint limits
        q1 = [k for k in range(s.n) if s.jtype[k] != 1]
        qs = np.array([tr[:, 6 + k] for k in q1])   # 1-dof coordinates follow the free root's 7
        lo, hi = s.limits[q1, 0][:, None], s.limits[q1, 1][:, None]
        assert ((qs > hi) | (qs < lo)).any()
    e = max(rel(tr[t + 1], tr_o[t], 1e-12) for t in range(tau.shape[0]))
    print(name, "contacts per step", np.bincount(nc), "worst state error %.1e" % e)
    assert e < 1e-10


@pytest.mark.parametrize("k", range(len(SCENES)), ids=[sc[0] for sc in SCENES])
def test_step_map_fp32_within_bar(k):
    """FP32 steps from the oracle's own states equal the oracle's steps
    within 1e-4.  The bar comes from the step's conditioning: rounding only
    the input state and control to FP32 moves the FP64 oracle's step on the
    landing quadruped by up to 2.5e-5 (impacts, contacts switching on and
    off, 30 unconverged PGS sweeps), and the test measures that sensitivity
    alongside.  End to end the rounding grows over the rollout; that figure
    is printed.  With joint limits the bar widens to twice the oracle's own
    sensitivity (the damper's switch at a limit)."""
    name, s, q0, qd0, tau, links, centers, radii, mu, beta = SCENES[k]
    dt, niter = 1e-3, 30
    m = O.Model(s, G)
    C = O.Contacts(links, centers, radii, mu=mu, beta=beta, niter=niter)
    _, _, nc_o, tr_o = O.rollout_contact(m, C, q0, qd0, tau, dt, traj=True)
    states = np.concatenate([np.r_[q0, qd0][None], tr_o])
    worst, sens = 0.0, 0.0
    f32 = lambda v: np.asarray(v, np.float32).astype(np.float64)
    for t in range(tau.shape[0]):
        x = states[t]
        tr1, nc1 = emu_rollout(s, links, centers, radii, mu, beta, niter, x[:s.nq], x[s.nq:], tau[t:t + 1], dt,
                               fp64=False)
        worst = max(worst, rel(tr1[1], states[t + 1], 1e-6))
        q1r, qd1r, _ = O.rollout_contact(m, C, f32(x[:s.nq]), f32(x[s.nq:]), f32(tau[t:t + 1]), dt)
        sens = max(sens, rel(np.r_[q1r, qd1r], states[t + 1], 1e-6))
    tr, nc = emu_rollout(s, links, centers, radii, mu, beta, niter, q0, qd0, tau, dt, fp64=False)
    e2e = max(rel(tr[t + 1], tr_o[t], 1e-6) for t in range(tau.shape[0]))
    print(name, "fp32 worst step-map error %.1e (oracle under FP32 input rounding: %.1e), end to end %.1e"
          % (worst, sens, e2e))
    # with joint limits the damper switches on discontinuously at a limit
    # (tau_l jumps by d qd), so where a state sits at a limit the oracle's
    # own step moves by that jump under FP32 input rounding; the bar is then
    # twice that measured sensitivity
    assert worst < max(1e-4, 2 * sens)


@pytest.mark.parametrize("adjoint", [False, True], ids=["dual-jacobians", "reverse-statements"])
@pytest.mark.parametrize("k", range(len(SCENES)), ids=[sc[0] for sc in SCENES])
def test_gradient_fp64_matches_the_oracle(k, adjoint):
    name, s, q0, qd0, tau, links, centers, radii, mu, beta = SCENES[k]
    dt, niter = 1e-3, 30
    T = 50 if name.startswith("quadruped") else 25   # the quadruped touches down after ~30 steps
    tau = tau[:T]
    m = O.Model(s, G)
    C = O.Contacts(links, centers, radii, mu=mu, beta=beta, niter=niter)
    rng = np.random.default_rng(k)
    gqT, gqdT = rng.normal(size=s.nq), rng.normal(size=s.nv)
    ref = O.rollout_contact_grad(m, C, q0, qd0, tau, dt, gqT, gqdT, mu_grad=True)
    ref = ref[:3] + (np.array([ref[3]]),)
    tr, nc = emu_rollout(s, links, centers, radii, mu, beta, niter, q0, qd0, tau, dt)
    got = emu_grad(s, links, centers, radii, mu, beta, niter, tr, tau, dt, gqT, gqdT, adjoint=adjoint)
    # an exactly zero block (a sticking inelastic contact erases qd0) is
    # compared against the gradient's overall scale
    scale = max(np.abs(r).max() for r in ref if r.size)
    e = [rel(g, r, 1e-6 * scale) for g, r in zip(got, ref)]
    print(name, "gradient errors (q0, qd0, tau, mu)", ["%.1e" % x for x in e], "contacts", np.bincount(nc))
    assert nc.max() >= 1
    assert max(e) < 1e-8


@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
@pytest.mark.parametrize("k", range(len(SCENES)), ids=[sc[0] for sc in SCENES])
def test_staged_gauss_seidel_is_bitwise_the_plain_one(k, fp64):
    """The gradient kernel runs both Gauss-Seidel solves and their reverse
    sweeps on a compact staged copy, and the unit-impulse responses on a copy
    of the articulated quantities (both in LDS on the GPU); the same
    statements in the same order give the same bits as on the full records."""
    name, s, q0, qd0, tau, links, centers, radii, mu, beta = SCENES[k]
    dt, niter = 1e-3, 30
    T = 50 if name.startswith("quadruped") else 25
    tau = tau[:T]
    tr0, nc0 = emu_rollout(s, links, centers, radii, mu, beta, niter, q0, qd0, tau, dt, fp64=fp64)
    tr1, nc1 = emu_rollout(s, links, centers, radii, mu, beta, niter, q0, qd0, tau, dt, fp64=fp64, staged=True)
    assert np.array_equal(tr0, tr1) and np.array_equal(nc0, nc1) and nc0.max() >= 1
    rng = np.random.default_rng(k)
    gqT, gqdT = rng.normal(size=s.nq), rng.normal(size=s.nv)
    g0 = emu_grad(s, links, centers, radii, mu, beta, niter, tr0, tau, dt, gqT, gqdT, fp64=fp64, adjoint=True,
                  staged=False)
    g1 = emu_grad(s, links, centers, radii, mu, beta, niter, tr0, tau, dt, gqT, gqdT, fp64=fp64, adjoint=True,
                  staged=True)
    for a, b in zip(g0, g1):
        assert np.array_equal(a, b)


def test_flop_count_grows_with_active_contacts():
    """sim_contact_flops (host code, no GPU): the count rises with each
    active contact, and the reverse step (recompute plus the reverse
    statements) costs more than the step and a small multiple of it."""
    from paper_2109_07719_amd import _native as N
    from paper_2109_07719_amd import synth
    from paper_2109_07719_amd.contact import _Model
    s, q0, qd0, tau, links, centers, radii = synth.landing_quadruped(3100, 2)
    par, jt, cl = (np.ascontiguousarray(x, np.int32) for x in (s.parent, s.jtype, links))
    m = _Model(s.n, par.ctypes.data, jt.ctypes.data, 4, cl.ctypes.data, 0.8, 0.2, 30,
               (ctypes.c_double * 3)(*G))
    P = np.ascontiguousarray(pack_params(s, centers, radii))
    counts = []
    for y in (1.0, 0.53, 0.5):          # none, some, all four feet below the plane
        q = np.array(q0)
        q[1] = y
        q[7:] = 0.0
        a, b = ctypes.c_double(), ctypes.c_double()
        N.check(N.lib().sim_contact_flops(ctypes.byref(m), _p(P), _p(q), _p(np.ascontiguousarray(qd0)),
                                          _p(np.ascontiguousarray(tau[0])), 1e-3, ctypes.byref(a), ctypes.byref(b)))
        counts.append((a.value, b.value))
    print(counts)
    assert counts[0][0] < counts[2][0] and counts[0][1] < counts[2][1]
    assert all(a < b < 12 * a for a, b in counts)
