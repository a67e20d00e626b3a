"""CPU-only checks of the C ABI library, the host logic and the GPU path's
per-link arithmetic (through the test-only host emulation)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from helpers import ball_tangent, emu_fd, emu_rollout_grad, rel
from paper_2109_07719_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# ---------------------------------------------------------------- C ABI library

def _declared_symbols():
    with open(os.path.join(ROOT, "include", "abadj.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^(?:int|void|const char \*)\s*\*?\s*(sim_\w+)\s*\(", text, re.M)))


def test_library_loads_and_exports_every_declared_symbol():
    from paper_2109_07719_amd import _native
    L = _native.lib()
    declared = _declared_symbols()
    assert len(declared) >= 9
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(_native.EXPORTED)


def _create(parent, jtype, n_sys_offsets, axis=None, mass=None, dtype=0):
    from paper_2109_07719_amd import _native as N
    nl = len(parent)
    arr = lambda a, t: np.ascontiguousarray(np.asarray(a, dtype=t))
    off = arr(n_sys_offsets, np.int32)
    par = arr(parent, np.int32)
    jt = arr(jtype, np.int32)
    E = arr(np.tile(np.eye(3).reshape(-1), nl), np.float64)
    r = arr(np.zeros(3 * nl), np.float64)
    ax = arr(np.tile([0, 0, 1.0], nl) if axis is None else axis, np.float64)
    m = arr(np.ones(nl) if mass is None else mass, np.float64)
    com = arr(np.zeros(3 * nl), np.float64)
    Ic = arr(np.tile([0.1, 0.1, 0.1, 0, 0, 0], nl), np.float64)
    g = arr([0, -9.81, 0], np.float64)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    topo = N.SimTopology(len(off) - 1, p(off), p(par), p(jt))
    prm = N.SimParams(p(E), p(r), p(ax), p(m), p(com), p(Ic), p(g))
    h = ctypes.c_void_p()
    rc = N.lib().sim_create(ctypes.byref(topo), ctypes.byref(prm), dtype, ctypes.byref(h))
    return rc, N.lib().sim_last_error().decode()


@pytest.mark.parametrize("parent,jtype,offsets,kw,code", [
    ([0, 0], [0, 0], [0, 2], {}, -2),                       # parent not < index
    ([-1, 1], [0, 0], [0, 2], {}, -2),                      # parent == index
    ([-1, -2], [0, 0], [0, 2], {}, -2),                     # parent < -1
    ([-1, 0], [0, 1], [0, 2], {}, -2),                      # free joint not at the root
    ([-1, -1], [1, 0], [0, 2], {}, -2),                     # free root plus a second base link
    ([-1, 0], [0, 7], [0, 2], {}, -2),                      # unknown joint type
    ([-1] * 65, [0] * 65, [0, 65], {}, -2),                  # more than 64 links
    ([-1, 0], [0, 0], [0, 2], {"axis": [0, 0, 2.0, 0, 0, 1.0]}, -2),  # non-unit axis
    ([-1, 0], [2, 2], [0, 2], {"axis": [0, 0, 1.0, 0, 0.5, 0]}, -2),  # non-unit prismatic axis
    ([-1, 0], [0, 0], [0, 2], {"mass": [1.0, 0.0]}, -2),    # non-positive mass
    ([-1, 0], [0, 0], [0, 2], {"mass": [1.0, np.nan]}, -2),  # non-finite parameter
    ([-1, 0], [0, 0], [1, 2], {}, -2),                      # link_offset[0] != 0
    ([-1, 0], [0, 0], [0, 2], {"dtype": 5}, -4),            # unsupported dtype
])
def test_create_rejects_invalid_input_before_touching_the_gpu(parent, jtype, offsets, kw, code):
    rc, msg = _create(parent, jtype, offsets, **kw)
    assert rc == code, msg
    assert msg


def test_null_arguments_are_rejected():
    from paper_2109_07719_amd import _native as N
    L = N.lib()
    h = ctypes.c_void_p()
    assert L.sim_create(None, None, 0, ctypes.byref(h)) == N.SIM_ERR_INVALID_ARG
    b = ctypes.c_size_t()
    assert L.sim_workspace_bytes(None, 10, 1, ctypes.byref(b)) == N.SIM_ERR_INVALID_ARG
    assert L.sim_forward(None, None, None, None, 1e-3, 1, 1, None, None, None, None, 0, None) == \
        N.SIM_ERR_INVALID_ARG
    assert L.sim_backward(None, None, 1e-3, 1, 1, None, None, None, None, None, None, None, None, None, 0, None) == \
        N.SIM_ERR_INVALID_ARG
    assert L.sim_aba(None, None, None, None, None, None) == N.SIM_ERR_INVALID_ARG
    f = ctypes.c_double()
    assert L.sim_flops(None, 0, ctypes.byref(f)) == N.SIM_ERR_INVALID_ARG
    n = ctypes.c_int()
    assert L.sim_status(None, None, ctypes.byref(n)) == N.SIM_ERR_INVALID_ARG
    t = N.SimTiling(1, 1, 1)
    assert L.sim_get_tiling(None, ctypes.byref(t)) == N.SIM_ERR_INVALID_ARG
    assert L.sim_set_tiling(None, ctypes.byref(t)) == N.SIM_ERR_INVALID_ARG
    assert L.sim_autotune(None, 1, 10, None, None, None) == N.SIM_ERR_INVALID_ARG
    L.sim_destroy(None)
    # contact solver: sizes and null arrays are rejected before any launch
    z = ctypes.c_size_t()
    assert L.sim_pgs_workspace_bytes(0, 4, 3, 10, None) == N.SIM_ERR_INVALID_ARG
    assert L.sim_pgs_workspace_bytes(0, 4, 17, 10, ctypes.byref(z)) == N.SIM_ERR_INVALID_ARG
    assert L.sim_pgs_workspace_bytes(0, 4, 0, 10, ctypes.byref(z)) == N.SIM_ERR_INVALID_ARG
    assert L.sim_pgs_workspace_bytes(7, 4, 3, 10, ctypes.byref(z)) == N.SIM_ERR_UNSUPPORTED_DTYPE
    assert L.sim_pgs_workspace_bytes(1, 4, 3, 10, ctypes.byref(z)) == N.SIM_OK and z.value == 11 * 3 * 4 * 8
    # from 13 rows the adjoint keeps its per-row coefficients after the sweep vectors
    assert L.sim_pgs_workspace_bytes(0, 4, 12, 10, ctypes.byref(z)) == N.SIM_OK and z.value == 11 * 12 * 4 * 4
    assert L.sim_pgs_workspace_bytes(0, 4, 13, 10, ctypes.byref(z)) == N.SIM_OK and z.value == 21 * 13 * 4 * 4
    assert L.sim_pgs_solve(0, 4, 3, 10, None, None, None, None, None, None, None, 0, None) == N.SIM_ERR_INVALID_ARG
    assert L.sim_pgs_solve(0, 4, 17, 10, None, None, None, None, None, None, None, 0, None) == N.SIM_ERR_INVALID_ARG
    assert L.sim_pgs_adjoint(0, 4, 3, 10, *([None] * 6), 0, *([None] * 6)) == N.SIM_ERR_INVALID_ARG
    assert b"sim_pgs_adjoint" in L.sim_last_error()
    # contact kernels' launch geometry: only the compiled systems-per-wave counts
    from paper_2109_07719_amd.contact import _Model, _Tiling
    par, jt, cl = (np.array(v, np.int32) for v in ([-1, 0], [N.SIM_JOINT_FREE, N.SIM_JOINT_REVOLUTE], [1]))
    sizes = [ctypes.c_int() for _ in range(4)]
    for tiling, ok in (((8, 16, 1), True), ((2, 4, 1), True), ((4, 8, 1), True), ((8, 16, 0), True),
                       ((3, 16, 1), False), ((8, 32, 1), False), ((16, 16, 1), False), ((8, 8, 0), False),
                       ((8, 16, 2), False)):
        t = _Tiling(*tiling)
        m = _Model(2, par.ctypes.data, jt.ctypes.data, 1, cl.ctypes.data, 0.5, 0.0, 10,
                   (ctypes.c_double * 3)(0.0, -9.81, 0.0), None, ctypes.addressof(t))
        rc = L.sim_contact_param_count(ctypes.byref(m), *[ctypes.byref(x) for x in sizes])
        assert rc == (N.SIM_OK if ok else N.SIM_ERR_INVALID_ARG), tiling
        if ok:
            assert [x.value for x in sizes] == [8, 7, 1, 2 * 25 + 4]
    assert b"tiling" in L.sim_last_error()
    m.tiling = None
    assert L.sim_contact_param_count(ctypes.byref(m), None, None, None, None) == N.SIM_OK
    # joint limits: checked like sim_params' (the free root's entry is not read)
    for lim, ok in (([9, 9, 9, 9, -0.5, 0.5, 100.0, 1.0], True), ([0, 0, 0, 0, 0.5, -0.5, 100.0, 1.0], False),
                    ([0, 0, 0, 0, -0.5, 0.5, -1.0, 1.0], False), ([0, 0, 0, 0, -0.5, np.inf, 1.0, 1.0], False)):
        la = np.array(lim, np.float64)
        m.limits = la.ctypes.data
        rc = L.sim_contact_param_count(ctypes.byref(m), None, None, None, None)
        assert rc == (N.SIM_OK if ok else N.SIM_ERR_INVALID_ARG), lim
    m.limits = None
    c = _Tiling()
    assert L.sim_contact_autotune(ctypes.byref(m), 0, 4, None, None, None, None, 1e-3, 10, None, ctypes.byref(c),
                                  None, None) == N.SIM_ERR_INVALID_ARG


# ---------------------------------------------------------------- generators

def test_generators_are_deterministic_and_shaped():
    a = synth.workload("chain7_4096", n_systems=3, T=20)
    b = synth.workload("chain7_4096", n_systems=3, T=20)
    assert np.array_equal(a.tau, b.tau) and np.array_equal(a.q0, b.q0)
    assert a.tau.shape == (20, 21) and a.total_dof == 21
    s = a.systems[0]
    assert list(s.parent) == [-1, 0, 1, 2, 3, 4, 5]
    assert np.allclose(s.r_T[1:], [0.5, 0, 0]) and np.allclose(s.com, [0.25, 0, 0])
    q = synth.workload("quad_1024", n_systems=2, T=3)
    assert (q.systems[0].nq, q.systems[0].nv, q.systems[0].nu) == (19, 18, 12)
    assert q.tau.shape == (3, 24)


def test_tree_generator_respects_size_and_depth():
    sizes, depths = [], []
    for i in range(200):
        s, _, _, _ = synth.tree_system(2000 + i, 1)
        sizes.append(s.n)
        depths.append(int(s.depth().max()))
        assert all(s.parent[k] < k for k in range(s.n))
        assert np.allclose(np.linalg.norm(s.axis, axis=1), 1)
    assert min(sizes) >= 6 and max(sizes) <= 40 and max(depths) <= 5
    assert 18 < np.mean(sizes) < 28


# ---------------------------------------------------------------- host emulation

@pytest.mark.parametrize("which", ["chain", "tree", "quad", "prismatic_tree", "cartpole", "telescoping_quad",
                                   "prismatic_chain", "ball_tree", "ball_quad"])
def test_lane_arithmetic_matches_oracle_fp64(which):
    """The per-link functions the kernels call, driven link by link on the
    host in FP64, reproduce the oracle's accelerations and rollout gradients
    to round-off (independent dense 6x6 arithmetic on the oracle side).  A
    ball joint's quaternion gradient is compared along the unit sphere (the
    oracle's radial part removed)."""
    if which == "chain":
        s, q0, qd0, tau = synth.chain_system(7, 1000, 120)
    elif which == "tree":
        s, q0, qd0, tau = synth.tree_system(2002, 120, random_frames=True)
    elif which == "quad":
        s, q0, qd0, tau = synth.quadruped_system(3003, 120)
    elif which == "prismatic_tree":
        s, q0, qd0, tau = synth.tree_system(2003, 120, random_frames=True, prismatic=0.4)
        assert (s.jtype == synth.PRISMATIC).sum() >= 3
    elif which == "cartpole":
        s, q0, qd0, tau = synth.cartpole_system(5, 120)
    elif which == "telescoping_quad":
        s, q0, qd0, tau = synth.telescoping_quadruped_system(3004, 120)
    elif which == "ball_tree":
        s, q0, qd0, tau = synth.ball_tree_system(2021, 120, random_frames=True, spherical=0.6)
        assert (s.jtype == synth.SPHERICAL).sum() >= 10
    elif which == "ball_quad":
        s, q0, qd0, tau = synth.ball_quadruped_system(3020, 120)
    else:
        s, q0, qd0, tau = synth.prismatic_chain_system(8, 1001, 120)
    m = O.Model(s)
    assert rel(emu_fd(s, q0, qd0, tau[0]), O.fd(m, q0, qd0, tau[0]), 1e-12) < 1e-13
    rng = np.random.default_rng(1)
    gqT, gqdT = rng.normal(size=s.nq), rng.normal(size=s.nv)
    a = emu_rollout_grad(s, q0, qd0, tau, 1e-3, gqT, gqdT)
    b = list(O.rollout_grad(m, q0, qd0, tau, 1e-3, gqT, gqdT))
    b[0] = ball_tangent(s, q0, b[0])
    for x, y in zip(a, b):
        assert rel(x, y, 1e-12) < 1e-11


@pytest.mark.parametrize("which", ["tree", "prismatic_tree", "telescoping_quad", "chain", "cartpole", "ball_tree",
                                   "ball_quad"])
def test_lane_arithmetic_frame_gradients_match_oracle_fp64(which):
    """The kernels' per-link placement and axis adjoints (transform adjoint
    G, motion-subspace adjoint, frame_bar_add), accumulated link by link on
    the host in FP64 and turned into the caller's frames, reproduce the
    oracle's dense placement and axis gradients to round-off."""
    from helpers import emu_rollout_grad
    if which == "tree":
        s, q0, qd0, tau = synth.tree_system(2014, 80, random_frames=True)
    elif which == "prismatic_tree":
        s, q0, qd0, tau = synth.tree_system(2015, 80, random_frames=True, prismatic=0.4)
    elif which == "telescoping_quad":
        s, q0, qd0, tau = synth.telescoping_quadruped_system(3011, 80)
    elif which == "chain":
        s, q0, qd0, tau = synth.chain_system(7, 1003, 80)
    elif which == "ball_tree":
        s, q0, qd0, tau = synth.ball_tree_system(2022, 80, random_frames=True, spherical=0.5)
    elif which == "ball_quad":
        s, q0, qd0, tau = synth.ball_quadruped_system(3021, 80)
    else:
        s, q0, qd0, tau = synth.cartpole_system(7, 80)
    m = O.Model(s)
    rng = np.random.default_rng(2)
    gqT, gqdT = rng.normal(size=s.nq), rng.normal(size=s.nv)
    got = emu_rollout_grad(s, q0, qd0, tau, 1e-3, gqT, gqdT, frame=True)[5]
    ref = O.rollout_grad_params(m, q0, qd0, tau, 1e-3, gqT, gqdT)[4]
    assert rel(got, ref, 1e-12) < 1e-11, (got, ref)


def test_lane_arithmetic_fp32_forward_dynamics_error():
    """The same per-link arithmetic in FP32 stays within the 1e-5 per-step
    bar on the chain workload (the GPU's arithmetic type)."""
    b = synth.round_to_f32(synth.workload("chain7_4096", n_systems=32, T=1))
    qo, vo, uo = b.offsets()
    errs = []
    for i, s in enumerate(b.systems):
        q, qd, tau = b.q0[qo[i]:qo[i + 1]], b.qd0[vo[i]:vo[i + 1]], b.tau[0, uo[i]:uo[i + 1]]
        ref = O.fd(O.Model(s), q, qd, tau)
        errs.append(rel(emu_fd(s, q, qd, tau, f32=True), ref))
    assert max(errs) < 1e-5, max(errs)


def _simulate_schedule(T, s):
    """Run a binomial checkpointing schedule symbolically: every ADJOINT
    must come in the order T-1, ..., 0 with the state at its own time."""
    from paper_2109_07719_amd import _native
    L = _native.lib()
    n, adv = ctypes.c_int(), ctypes.c_longlong()
    assert L.sim_checkpoint_schedule(T, s, None, 0, ctypes.byref(n), ctypes.byref(adv)) == 0
    buf = (ctypes.c_int32 * (2 * max(n.value, 1)))()
    assert L.sim_checkpoint_schedule(T, s, buf, n.value, ctypes.byref(n), ctypes.byref(adv)) == 0
    acts = [(buf[2 * i], buf[2 * i + 1]) for i in range(n.value)]
    slots = {0: 0}
    cur, adjoints, advanced = None, [], 0
    for op, arg in acts:
        what, slot = op & 7, op >> 3
        if what == 0:
            assert slots.get(slot) == arg, (T, s, "restore of a slot that does not hold that time")
            cur = arg
        elif what == 1:
            assert cur is not None and arg > 0
            cur += arg
            advanced += arg
        elif what == 2:
            assert 1 <= slot <= s and cur is not None
            slots[slot] = cur
        else:
            assert what == 3 and cur == arg, (T, s, "adjoint away from its state")
            adjoints.append(arg)
    assert adjoints == list(range(T - 1, -1, -1))
    assert advanced == adv.value
    return advanced


def test_binomial_schedule_reverses_every_step_in_order():
    for T in range(0, 40):
        for s in range(1, 6):
            _simulate_schedule(T, s)


def test_binomial_schedule_recompute_bound():
    """With s snapshots and repetition number r (the least r with
    C(s + r, s) >= T), no step is advanced more than r times, so the schedule
    advances at most r * T steps; one snapshot gives the quadratic count."""
    from math import comb
    for T, s in [(1000, 4), (5000, 10), (50000, 16), (50000, 3), (200, 1)]:
        r = next(r for r in range(1, T + 1) if comb(s + r, s) >= T)
        adv = _simulate_schedule(T, s)
        assert adv <= r * T, (T, s, adv, r)
        if s == 1:
            assert adv == T * (T - 1) // 2


def test_fast_free_base_keeps_fp32_joint_accelerations():
    """The kernels evaluate a free root's ABA in the frame that moves with
    its linear velocity (an exact Galilean shift), so in FP32 the joint
    accelerations do not lose digits when the base moves fast (a long free
    fall reaches hundreds of m/s); the emulation of the same per-link math
    against the FP64 oracle, at rest and at 300 and 3000 m/s."""
    r = lambda x: x.astype(np.float32).astype(np.float64)
    for speed in (0.0, 300.0, 3000.0):
        for seed in range(3000, 3004):
            s, q0, qd0, tau = synth.quadruped_system(seed, 1)
            s = synth.round_to_f32(synth.make_batch([(s, q0, qd0, tau)], 1e-3)).systems[0]
            rng = np.random.default_rng(seed)
            q = q0.copy()
            qt = rng.normal(size=4)
            q[3:7] = qt / np.linalg.norm(qt)
            q[7:] = rng.normal(0, 0.5, 12)
            qd = rng.normal(0, 1, 18)
            d = rng.normal(size=3)
            qd[3:6] = speed * d / np.linalg.norm(d)
            q, qd, t = r(q), r(qd), r(tau[0])
            ref = O.fd(O.Model(s), q, qd, t)
            got = emu_fd(s, q, qd, t, f32=True)
            assert np.linalg.norm(got[6:] - ref[6:]) < 2e-6 * np.linalg.norm(ref[6:]), (speed, seed)
            assert np.linalg.norm(got[:6] - ref[:6]) < 2e-6 * np.linalg.norm(ref[:6]), (speed, seed)


# ---------------------------------------------------------------- forward kinematics helper

def test_link_points_match_world_kinematics_with_prismatic_joints():
    """The loss-side FK helper (revolute, prismatic, spherical and free-root
    links) against the independent world-frame kinematics of the
    Newton-Euler reference, on trees with random frames, prismatic and ball
    joints, a cart-pole and quadrupeds (one on ball hips); an unknown joint
    type is rejected instead of mis-handled."""
    import torch
    from dyn_ref import kinematics
    from paper_2109_07719_amd.fk import LinkPoints
    rng = np.random.default_rng(5)
    draws = [synth.tree_system(2100 + i, 1, random_frames=True, prismatic=0.4) for i in range(4)]
    draws += [synth.cartpole_system(7, 1), synth.quadruped_system(3007, 1), synth.prismatic_chain_system(5, 9, 1)]
    draws += [synth.ball_tree_system(2200 + i, 1, random_frames=True, spherical=0.5) for i in range(2)]
    draws += [synth.ball_quadruped_system(3008, 1)]
    for sys_, q0, qd0, _ in draws:
        q = np.asarray(q0, dtype=np.float64) + rng.normal(0, 0.3, len(q0))
        qo = 0
        for i in range(sys_.n):
            if sys_.jtype[i] == 1:
                q[qo + 3:qo + 7] /= np.linalg.norm(q[qo + 3:qo + 7])
            elif sys_.jtype[i] == 3:
                q[qo:qo + 4] /= np.linalg.norm(q[qo:qo + 4])
            qo += 7 if sys_.jtype[i] == 1 else 4 if sys_.jtype[i] == 3 else 1
        pts = rng.normal(0, 0.3, (sys_.n, 3))
        R, o, *_ = kinematics(sys_, q, np.zeros(sys_.nv), np.zeros(sys_.nv), (0.0, -9.81, 0.0))
        for link in range(sys_.n):
            fk = LinkPoints([sys_], [link], pts[link:link + 1], dtype=torch.float64, device="cpu")
            got = fk(torch.tensor(q))[0].numpy()
            ref = o[link] + R[link] @ pts[link]
            assert np.allclose(got, ref, rtol=0, atol=1e-12), (link, got, ref)
    bad, *_ = synth.tree_system(2200, 1)
    bad = synth.replace(bad, jtype=np.where(np.arange(bad.n) == bad.n - 1, 7, bad.jtype).astype(np.int32))
    with pytest.raises(ValueError, match="joint type 7"):
        LinkPoints([bad], [bad.n - 1], [[0.5, 0.0, 0.0]], dtype=torch.float64, device="cpu")
