"""GPU parity of rollouts with contact inside the step and of their
gradient (Sec. 4.1 "Collision resolution"), through the C ABI
(sim_contact_rollout, sim_contact_rollout_grad), against the FP64 oracle:

* FP64 trajectories and contact counts element by element on sampled
  systems of a 256-quadruped landing batch and of a 64-tree batch (prismatic
  joints, random frames), to round-off;
* FP64 gradients (q0, qd0, tau and the friction coefficient mu) against the
  oracle's, to round-off, through touchdown;
* FP32: the GPU's step from its own states against the oracle's step,
  within the bar the step's conditioning sets (1e-4, see the host test), and
  the FP32 rollout's gradient (recomputed and reversed in FP64) against the
  oracle's gradient along the GPU's own trajectory;
* edge cases: no contact spheres (the plain step), an empty batch, invalid
  models;
* every launch geometry (systems per wave) gives the same bits, and the
  autotuner picks one of them;
* joint limits inside the step (FP64 states and gradients to round-off);
* the benchmark batch (4096 quadrupeds, 1000 steps) on sampled systems:
  steps and the full-horizon gradient along the GPU trajectory.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import contact_cases as CC
import dyn_ref as R
import oracle as O
from helpers import TOL_GRAD_F32, rel
from paper_2109_07719_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"
G = (0.0, -9.81, 0.0)
MU, BETA, NITER, DT = 0.8, 0.2, 30, 1e-3


def _world_point(s, q, link, c):
    Rs, o, *_ = R.kinematics(s, q, np.zeros(s.nv), np.zeros(s.nv), np.array(G))
    return o[link] + Rs[link] @ c


def quad_batch(B, T, seed0=3100):
    draws = [CC.landing_quadruped(seed0 + i, T) for i in range(B)]
    return draws


def tree_batch(B, T, seed=2003):
    """One tree topology; masses, inertias, COMs, sphere centres and radii
    and the states vary per system."""
    base = CC.grounded_tree(seed, T)
    out = []
    for i in range(B):
        rng = np.random.default_rng(100 + i)
        s, q0, qd0, tau, links, centers, radii = CC.grounded_tree(seed, T)
        s.mass = s.mass * rng.uniform(0.8, 1.25, s.n)
        s.com = s.com + rng.normal(0, 0.02, s.com.shape)
        q0 = q0 + rng.normal(0, 0.05, q0.shape)
        centers = centers + rng.normal(0, 0.02, centers.shape)
        s = CC.lower_to_ground(s, q0, links, centers, radii, _world_point, rng.uniform(1e-3, 5e-3))
        out.append((s, q0, qd0, tau, links, centers, radii))
    assert all(np.array_equal(d[0].parent, base[0].parent) for d in out)
    return out


def _gpu(draws, dtype, T, mu=MU, beta=BETA, niter=NITER):
    from paper_2109_07719_amd.contact import ContactBatch
    cb = ContactBatch([d[0] for d in draws], draws[0][4], [d[5] for d in draws], [d[6] for d in draws], mu=mu,
                      beta=beta, niter=niter, gravity=G, dtype=dtype)
    f = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)
    q0 = f(np.stack([d[1] for d in draws], axis=1))
    qd0 = f(np.stack([d[2] for d in draws], axis=1))
    tau = f(np.stack([d[3][:T] for d in draws], axis=2))
    return cb, q0, qd0, tau


def _oracle(d, mu=MU, beta=BETA, niter=NITER):
    s, q0, qd0, tau, links, centers, radii = d
    return O.Model(s, G), O.Contacts(links, centers, radii, mu=mu, beta=beta, niter=niter)


def _r32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _oracle32(d, mu=MU, beta=BETA, niter=NITER):
    """The oracle's model of an FP32 batch: parameters, sphere geometry,
    gravity and the solver constants rounded to FP32 as the GPU holds them."""
    s, q0, qd0, tau, links, centers, radii = d
    s32 = synth.System(parent=s.parent, jtype=s.jtype, E_T=_r32(s.E_T), r_T=_r32(s.r_T), axis=_r32(s.axis),
                       mass=_r32(s.mass), com=_r32(s.com), Ic=_r32(s.Ic))
    return (O.Model(s32, _r32(G)),
            O.Contacts(links, _r32(centers), _r32(radii), mu=float(_r32(mu)), beta=float(_r32(beta)), niter=niter))


def _oracle_grad_along(m, C, nq, traj_i, tau_i, dt, gqT, gqdT):
    """The oracle's rollout gradient along a given trajectory: its one-step
    gradient at every stored state x^t (traj_i [T + 1, nq + nv]), applied
    backwards in time.  Returns gq0, gqd0, gtau [T, nu], gmu."""
    T = tau_i.shape[0]
    gq, gqd = np.asarray(gqT, np.float64), np.asarray(gqdT, np.float64)
    gtau = np.zeros(tau_i.shape)
    gmu = 0.0
    for t in range(T - 1, -1, -1):
        x = traj_i[t]
        gq, gqd, gt, gm = O.rollout_contact_grad(m, C, x[:nq], x[nq:], tau_i[t:t + 1], dt, gq, gqd, mu_grad=True)
        gtau[t] = gt[0]
        gmu += gm
    return gq, gqd, gtau, gmu


@pytest.mark.parametrize("which", ["quadrupeds", "trees"])
def test_rollout_fp64_round_off(which):
    T = 100 if which == "quadrupeds" else 40
    draws = quad_batch(256, T) if which == "quadrupeds" else tree_batch(64, T)
    print("case", which, "B", len(draws), "T", T, flush=True)
    cb, q0, qd0, tau = _gpu(draws, torch.float64, T)
    qT, qdT, tr, nc = cb.rollout(q0, qd0, tau, DT, traj=True, counts=True)
    torch.cuda.synchronize()
    tr, nc = tr.cpu().numpy(), nc.cpu().numpy()
    worst, touched = 0.0, 0
    for i in range(0, len(draws), max(1, len(draws) // 16)):
        m, C = _oracle(draws[i])
        d = draws[i]
        _, _, nc_o, tr_o = O.rollout_contact(m, C, d[1], d[2], d[3][:T], DT, traj=True)
        assert np.array_equal(nc[:, i], nc_o), i
        touched += int(nc_o.max() >= 1)
        worst = max(worst, max(rel(tr[t + 1, :, i], tr_o[t], 1e-12) for t in range(T)))
    print("worst state error %.1e, sampled systems in contact %d" % (worst, touched))
    assert touched >= 8 and worst < 1e-10
    assert np.array_equal(qT.cpu().numpy(), tr[-1, :cb.nq]) and np.array_equal(qdT.cpu().numpy(), tr[-1, cb.nq:])


@pytest.mark.parametrize("which", ["quadrupeds", "trees"])
def test_gradient_fp64_round_off(which):
    T = 50 if which == "quadrupeds" else 25
    draws = quad_batch(64, T) if which == "quadrupeds" else tree_batch(32, T)
    print("case", which, "B", len(draws), "T", T, flush=True)
    cb, q0, qd0, tau = _gpu(draws, torch.float64, T)
    qT, qdT, tr = cb.rollout(q0, qd0, tau, DT)
    rng = np.random.default_rng(9)
    gqT = torch.tensor(rng.normal(size=(cb.nq, cb.B)), dtype=torch.float64, device=DEV)
    gqdT = torch.tensor(rng.normal(size=(cb.nv, cb.B)), dtype=torch.float64, device=DEV)
    g = [x.cpu().numpy() for x in cb.grad(tr, tau, DT, gqT, gqdT, mu_grad=True)]
    worst = 0.0
    for i in (0, 7, len(draws) // 2, len(draws) - 1):
        m, C = _oracle(draws[i])
        d = draws[i]
        ref = O.rollout_contact_grad(m, C, d[1], d[2], d[3][:T], DT, gqT[:, i].cpu().numpy(),
                                     gqdT[:, i].cpu().numpy(), mu_grad=True)
        ref = ref[:3] + (np.array([ref[3]]),)
        scale = max(np.abs(r).max() for r in ref)
        got = (g[0][:, i], g[1][:, i], g[2][:, :, i], g[3][i:i + 1])
        worst = max(worst, *[rel(a, b, 1e-6 * scale) for a, b in zip(got, ref)])
    print("worst gradient error %.1e" % worst)
    assert worst < 1e-8


def test_fp32_step_map_and_gradient():
    T = 60
    draws = quad_batch(128, T)
    print("case quadrupeds fp32 B 128 T", T, flush=True)
    cb, q0, qd0, tau = _gpu(draws, torch.float32, T)
    qT, qdT, tr = cb.rollout(q0, qd0, tau, DT)
    trn = tr.double().cpu().numpy()
    worst = 0.0
    for i in (0, 33, 77, 127):
        m, C = _oracle32(draws[i])
        tau_i = tau[:, :, i].double().cpu().numpy()
        for t in range(0, T, 3):
            x = trn[t, :, i]
            q1, qd1, _, _ = O.step_contact(m, C, x[:cb.nq], x[cb.nq:], tau_i[t], DT)
            worst = max(worst, rel(trn[t + 1, :, i], np.r_[q1, qd1], 1e-6))
    print("fp32 worst step-map error %.1e" % worst)
    assert worst < 1e-4
    # the gradient of the whole FP32 rollout (fall and touchdown) against the
    # oracle's gradient along the GPU's own trajectory
    rng = np.random.default_rng(4)
    gqT = torch.tensor(rng.normal(size=(cb.nq, cb.B)), dtype=torch.float32, device=DEV)
    gqdT = torch.tensor(rng.normal(size=(cb.nv, cb.B)), dtype=torch.float32, device=DEV)
    g = [x.double().cpu().numpy() for x in cb.grad(tr, tau, DT, gqT, gqdT, mu_grad=True)]
    worst_g = _along_errors(cb, draws, trn, tau, gqT, gqdT, g, (0, 33, 77, 127))
    print("fp32 worst gradient error along the GPU trajectory %.1e" % worst_g)
    assert worst_g < TOL_CONTACT_ALONG


# The FP32 contact gradient recomputes and reverses every step in FP64 from
# the GPU's own FP32 states, with the constants the forward rollout used; the
# oracle's one-step gradients at the same states, chained backwards, differ
# from it only by FP64 rounding of two different evaluation orders (and by
# the FP32 rounding of the outputs, 6e-8).  Over the 60-step landing that
# keeps them within 1e-6.  Over 1000 steps of persistent contact the
# backward recursion amplifies those roundings (measured 1e-5 to 2e-5 on
# the benchmark batch); there the FP32 gradient bar applies.
TOL_CONTACT_ALONG = 1e-6


def _along_errors(cb, draws, trn, tau, gqT, gqdT, g, sample):
    """Largest per-system error (q0, qd0, tau, mu) of the GPU gradient g
    against the oracle's gradient along the GPU trajectory trn."""
    dt32 = float(_r32(DT))
    worst = 0.0
    for i in sample:
        m, C = _oracle32(draws[i])
        ref = _oracle_grad_along(m, C, cb.nq, trn[:, :, i], tau[:, :, i].double().cpu().numpy(), dt32,
                                 gqT[:, i].double().cpu().numpy(), gqdT[:, i].double().cpu().numpy())
        got = (g[0][:, i], g[1][:, i], g[2][:, :, i], g[3][i])
        scale = max(np.abs(r).max() for r in ref[:3])
        e = [rel(a, b, 1e-6 * scale) for a, b in zip(got, ref)]
        print(f"system {i}: gradient errors along the GPU trajectory (q0, qd0, tau, mu) "
              + " ".join("%.1e" % x for x in e), flush=True)
        worst = max(worst, *e)
    return worst


def test_edge_cases():
    from paper_2109_07719_amd import _native as N
    from paper_2109_07719_amd.contact import ContactBatch
    # no spheres: the plain step of the oracle
    draws = [CC.landing_quadruped(3100 + i, 20) for i in range(3)]
    draws = [(d[0], d[1], d[2], d[3], np.zeros(0, np.int32), np.zeros((0, 3)), np.zeros(0)) for d in draws]
    cb, q0, qd0, tau = _gpu(draws, torch.float64, 20)
    qT, qdT, tr, nc = cb.rollout(q0, qd0, tau, DT, counts=True)
    assert not nc.any()
    m = O.Model(draws[1][0], G)
    qT_o, qdT_o = O.rollout(m, draws[1][1], draws[1][2], draws[1][3][:20], DT)
    assert rel(qT[:, 1].cpu().numpy(), qT_o, 1e-12) < 1e-12 and rel(qdT[:, 1].cpu().numpy(), qdT_o, 1e-12) < 1e-12
    # empty batch
    cb0, *_ = _gpu(draws[:1], torch.float64, 20)
    cb0.B = 0
    z = lambda *sh: torch.zeros(sh, dtype=torch.float64, device=DEV)
    out = cb0.rollout(z(cb0.nq, 0), z(cb0.nv, 0), z(5, cb0.nu, 0), DT, traj=False)
    assert out[0].shape == (cb0.nq, 0)
    # invalid models
    s = draws[0][0]
    bad = synth.System(parent=s.parent, jtype=np.where(np.arange(s.n) == 2, synth.SPHERICAL, s.jtype).astype(np.int32),
                       E_T=s.E_T, r_T=s.r_T, axis=s.axis, mass=s.mass, com=s.com, Ic=s.Ic)
    with pytest.raises(N.SimError):
        ContactBatch([bad], [3], [[[0, 0, 0]]], [[0.03]], dtype=torch.float64)
    with pytest.raises(N.SimError):
        ContactBatch([s], [3, 6, 9, 12, 3], [[[0, 0, 0]] * 5], [[0.03] * 5], dtype=torch.float64)
    big, *_ = synth.tree_system(5, 1, nmin=17, nmax=17)
    with pytest.raises(N.SimError):
        ContactBatch([big], [1], [[[0, 0, 0]]], [[0.03]], dtype=torch.float64)


def test_joint_limits_fp64_round_off():
    """Joint limits inside the step with contact (one set shared by the
    batch, tight around the start pose so the legs run into them): FP64
    states, contact counts and gradients against the oracle's."""
    from dataclasses import replace
    T = 50
    draws = quad_batch(32, T)
    lim = synth.with_joint_limits(draws[0][:4], 77, half_range=(0.002, 0.02))[0].limits
    draws = [(replace(d[0], limits=lim),) + tuple(d[1:]) for d in draws]
    print("case limits B", len(draws), "T", T, flush=True)
    cb, q0, qd0, tau = _gpu(draws, torch.float64, T)
    qT, qdT, tr, nc = cb.rollout(q0, qd0, tau, DT, counts=True)
    rng = np.random.default_rng(12)
    gqT = torch.tensor(rng.normal(size=(cb.nq, cb.B)), dtype=torch.float64, device=DEV)
    gqdT = torch.tensor(rng.normal(size=(cb.nv, cb.B)), dtype=torch.float64, device=DEV)
    g = [x.cpu().numpy() for x in cb.grad(tr, tau, DT, gqT, gqdT, mu_grad=True)]
    trn, ncn = tr.cpu().numpy(), nc.cpu().numpy()
    worst_x, worst_g, hit = 0.0, 0.0, False
    q1 = [k for k in range(draws[0][0].n) if draws[0][0].jtype[k] != 1]
    for i in (0, 9, 20, 31):
        m, C = _oracle(draws[i])
        d = draws[i]
        _, _, nc_o, tr_o = O.rollout_contact(m, C, d[1], d[2], d[3][:T], DT, traj=True)
        assert np.array_equal(ncn[:, i], nc_o), i
        worst_x = max(worst_x, max(rel(trn[t + 1, :, i], tr_o[t], 1e-12) for t in range(T)))
        qs = trn[:, [6 + k for k in q1], i]
        hit |= bool(((qs > lim[q1, 1]) | (qs < lim[q1, 0])).any())
        ref = O.rollout_contact_grad(m, C, d[1], d[2], d[3][:T], DT, gqT[:, i].cpu().numpy(),
                                     gqdT[:, i].cpu().numpy(), mu_grad=True)
        ref = ref[:3] + (np.array([ref[3]]),)
        scale = max(np.abs(r).max() for r in ref)
        got = (g[0][:, i], g[1][:, i], g[2][:, :, i], g[3][i:i + 1])
        worst_g = max(worst_g, *[rel(a, b, 1e-6 * scale) for a, b in zip(got, ref)])
    print("limits: worst state error %.1e, worst gradient error %.1e" % (worst_x, worst_g))
    assert hit and ncn.max() >= 2
    assert worst_x < 1e-10 and worst_g < 1e-8


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_every_tiling_gives_the_same_bits(dtype):
    """Each system is one lane whatever the launch geometry, so every
    systems-per-wave choice of the rollout and of the gradient gives the same
    trajectories, contact counts and gradients bit for bit; the autotuner
    returns one of them.  37 systems: a ragged last workgroup at every
    geometry."""
    T = 40
    draws = quad_batch(37, T)
    print("case tilings", dtype, "B", len(draws), "T", T, flush=True)
    cb, q0, qd0, tau = _gpu(draws, dtype, T)
    rng = np.random.default_rng(4)
    gqT = torch.tensor(rng.normal(size=(cb.nq, cb.B)), dtype=dtype, device=DEV)
    gqdT = torch.tensor(rng.normal(size=(cb.nv, cb.B)), dtype=dtype, device=DEV)
    ref = None
    for rs, gs, gl in ((8, 16, 1), (4, 8, 1), (2, 4, 1), (8, 4, 1), (2, 16, 1), (8, 16, 0)):
        cb.set_tiling(rs, gs, gl)
        qT, qdT, tr, nc = cb.rollout(q0, qd0, tau, DT, counts=True)
        g = cb.grad(tr, tau, DT, gqT, gqdT, mu_grad=True)
        out = [x.cpu().numpy() for x in (qT, qdT, tr, nc) + tuple(g)]
        if ref is None:
            ref = out
            assert int(out[3].max()) >= 2
        else:
            for a, b in zip(out, ref):
                assert np.array_equal(a, b), (rs, gs, gl)
    tune = cb.autotune(q0, qd0, tau[:10], DT)
    print("autotune", tune)
    assert tune["rollout_systems_per_wave"] in (8, 4, 2) and tune["grad_systems_per_wave"] in (16, 8, 4)
    assert tune["grad_lds"] in (0, 1)
    assert tune["rollout_ms_per_probe_step"] > 0 and tune["grad_ms_per_probe_step"] > 0
    assert cb.tiling == {k: tune[k] for k in ("rollout_systems_per_wave", "grad_systems_per_wave", "grad_lds")}
    qT, qdT, tr = cb.rollout(q0, qd0, tau, DT)
    assert np.array_equal(tr.cpu().numpy(), ref[2])


def test_benchmark_batch_sampled():
    """4096 landing quadrupeds, 1000 steps (1 s: fall, touchdown, then the
    legs fold under random torques with 2-4 feet on the ground; only the feet
    carry spheres), FP32 in one launch each way; sampled systems' GPU steps
    against the oracle's, and the gradient is finite."""
    T, B = 1000, 4096
    draws = quad_batch(B, T, seed0=50000)
    print("case benchmark batch B", B, "T", T, flush=True)
    cb, q0, qd0, tau = _gpu(draws, torch.float32, T)
    qT, qdT, tr, nc = cb.rollout(q0, qd0, tau, DT, counts=True)
    g = cb.grad(tr, tau, DT, 2 * qT, qdT.clone(), mu_grad=True)
    torch.cuda.synchronize()
    assert all(torch.isfinite(x).all() for x in g)
    ncn = nc.cpu().numpy()
    assert (ncn[-100:].min(axis=0) >= 1).mean() > 0.9, "feet stay in contact over the last 0.1 s"
    trn = tr[:, :, ::512].double().cpu().numpy()
    worst = 0.0
    for k, i in enumerate(range(0, B, 512)):
        m, C = _oracle(draws[i])
        tau_i = tau[:, :, i].double().cpu().numpy()
        for t in range(0, T, 97):
            x = trn[t, :, k]
            q1, qd1, _, _ = O.step_contact(m, C, x[:cb.nq], x[cb.nq:], tau_i[t], DT)
            worst = max(worst, rel(trn[t + 1, :, k], np.r_[q1, qd1], 1e-6))
    print("benchmark batch: fp32 worst sampled step-map error %.1e" % worst)
    assert worst < 1e-4
    # the gradient of the full 1000-step rollout along the GPU trajectory
    sample = list(range(0, B, 512))
    gn = [x.double().cpu().numpy() for x in g]
    gn = [gn[0][:, sample], gn[1][:, sample], gn[2][:, :, sample], gn[3][sample]]
    gq, gqd = (2 * qT)[:, sample], qdT[:, sample]
    worst_g = _along_errors(cb, [draws[i] for i in sample], trn, tau[:, :, sample], gq, gqd, gn,
                            list(range(len(sample))))
    print("benchmark batch: fp32 worst gradient error along the GPU trajectory %.1e" % worst_g)
    assert worst_g < TOL_GRAD_F32
