#!/usr/bin/env python
"""Benchmark of the hot path on one MI355X.

One "step" is one pass of the whole path over the batch: a T-step forward
rollout that checkpoints the initial state of every step, then the adjoint
rollout that recomputes each step and back-propagates (Sec. 4.1-4.2).
Default workload: 4096 fixed-base 7-DOF revolute chains, dt = 1e-3,
T = 5000, FP32, checkpoint every step, forward and adjoint captured in one
HIP graph (the timed step; each is also captured alone for the per-kernel
split).  Inputs are resident in HBM before the timed region.

Prints one JSON line: fwd+adjoint DOF-steps/s (value), the plain-forward
rate beside it, the gradient error against the FP64 oracle on sampled
systems, a roofline entry for the dominant (adjoint) kernel and the FP64
CPU oracle timed on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "chains_2048": "2048 fixed-base revolute chains of 5-50 links, dt=1e-3, T=1000, trajectory optimisation "
                   "of tau by Adam on ||end-effector - target||^2 + 1e-4 ||tau||^2",
    "chain7_4096": "4096 fixed-base 7-DOF revolute chains (z axes, links 0.5 m), dt=1e-3, T=5000, "
                   "checkpoint every step, forward+adjoint",
    "trees_8192": "8192 fixed-base uneven revolute trees (6-40 links, depth<=6), dt=5e-4, T=2000, "
                  "checkpoint every step, forward+adjoint",
    "quad_1024": "1024 free-floating quadrupeds (base + 4x3 revolute), dt=1e-3, T=50000, "
                 "checkpoint every step, forward+adjoint",
    "trees_prismatic_8192": "the 8192 uneven trees of trees_8192 with each joint prismatic with probability 0.3, "
                            "dt=5e-4, T=2000, checkpoint every step, forward+adjoint",
    "ball_quad_1024": "1024 free-floating quadrupeds on ball hips (base + 4x(ball + 2 revolute), n_v = 26), "
                      "dt=1e-3, T=2000, checkpoint every step, forward+adjoint",
}
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 vector peak (dual-issue); 78.6 without packed issue
FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector peak


KERNEL_SOURCES = ("csrc/spatial.h", "csrc/aba_lane.h", "csrc/dual.h", "csrc/abadj_device.h", "csrc/abadj_kernels.hip",
                  "csrc/abadj_kernels_bwd.hip", "csrc/abadj_kernels_bwd64.hip", "csrc/abadj_kernels_chain.hip",
                  "_build.py")


CONTACT_SOURCES = ("csrc/spatial.h", "csrc/dual.h", "csrc/contact_step.h", "csrc/contact_adjoint.h",
                   "csrc/contact.hip", "_build.py")


def _hash(sources):
    h = hashlib.sha256()
    for n in sources:
        with open(os.path.join(ROOT, "paper_2109_07719_amd", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_source_hash():
    """Hash of everything that decides the articulated-body kernels' machine
    code (their device sources and the build options)."""
    return _hash(KERNEL_SOURCES)


def contact_source_hash():
    """The same for the kernels with contact inside the step."""
    return _hash(CONTACT_SOURCES)


def traffic_entry(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    runs, if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def progress(msg):
    """A progress line on stderr (the legs of a long run report as they end)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def host_threads():
    """Host threads for the CPU legs: the cores this process may run on,
    capped by the host's thread budget for the job (OMP_NUM_THREADS, which
    the GPU host sets to its CPU share per GPU)."""
    avail = len(os.sched_getaffinity(0))
    cap = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return max(1, min(avail, cap) if cap > 0 else avail), avail


def host_cpu():
    import platform
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return cpu


def along_errors(batch, grads, idx, trajs, threads, window=2000):
    """Gradient errors of the GPU result on sampled systems against the FP64
    oracle's adjoint sweep along the GPU's own trajectory (its states used
    as the per-step checkpoints).  Returns per-system tuples (state/control
    error, parameter-gradient error, largest exact gradient entry, error of
    the control gradient over the last `window` steps, elementwise error of
    the control gradient) or None for a diverged rollout."""
    import oracle as O

    qo, vo, uo = batch.offsets()
    gq0, gqd0, gtau, gparam, gframe = grads
    lo = np.cumsum([0] + [s.n for s in batch.systems])
    window = min(batch.T, window)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-6))

    def along(k):
        i = idx[k]
        if not np.isfinite(trajs[k]).all():
            return None   # the rollout itself diverged (see the note)
        m = O.Model(batch.systems[i], batch.gravity)
        x0 = np.r_[batch.q0[qo[i]:qo[i + 1]], batch.qd0[vo[i]:vo[i + 1]]]
        states = np.concatenate([x0[None], trajs[k][:-1]])
        nqi = qo[i + 1] - qo[i]
        tau = np.asarray(batch.tau[:, uo[i]:uo[i + 1]], dtype=np.float64)
        g = list(O.adjoint_along_params(m, states, tau, batch.dt, 2 * trajs[k][-1, :nqi],
                                        np.zeros(vo[i + 1] - vo[i])))
        g[0] = O.ball_tangent(batch.systems[i], x0[:nqi], g[0])  # ball quaternions: along the sphere
        size = max(float(np.abs(x).max()) if x.size else 0.0 for x in g[:3])
        gt = gtau[:, uo[i]:uo[i + 1]]
        e_win = rel(gt[-window:], g[2][-window:]) if gt.size else 0.0
        e_elem = float(np.abs(gt - g[2]).max() / max(np.abs(g[2]).max(), 1e-30)) if gt.size else 0.0
        e_par = (max(rel(gparam[lo[i]:lo[i + 1]], g[3]), rel(gframe[lo[i]:lo[i + 1]], g[4]))
                 if gparam is not None else float("nan"))
        return (max(rel(gq0[qo[i]:qo[i + 1]], g[0]), rel(gqd0[vo[i]:vo[i + 1]], g[1]), rel(gt, g[2])),
                e_par, size, e_win, e_elem)

    return O.map_threads(along, range(len(idx)), threads=threads)


def summarise_along(both, window):
    """Statistics of along_errors over the sample."""
    diverged = sum(r is None for r in both)
    # the exact gradient of a long chaotic rollout can exceed the FP32 range
    fp32_max = float(np.finfo(np.float32).max)
    fits = [r for r in both if r is not None and r[2] < 1e-3 * fp32_max]
    beyond = sum(r is not None and r[2] >= 1e-3 * fp32_max for r in both)
    e_along = np.asarray([r[0] for r in fits] or [float("nan")])
    e_elem = [r[4] for r in fits] or [float("nan")]
    e_window = [r[3] for r in both if r is not None and np.isfinite(r[3])] or [float("nan")]
    return {"along_gpu_trajectory_max": float(e_along.max()),
            "along_gpu_trajectory_median": float(np.median(e_along)),
            "along_gpu_trajectory_p99": float(np.percentile(e_along, 99)),
            "along_gpu_trajectory_frac_above_1e-3": float(np.mean(e_along > 1e-3)),
            "along_gpu_trajectory_frac_above_1e-4": float(np.mean(e_along > 1e-4)),
            "gtau_elementwise_along_gpu_trajectory_max": float(max(e_elem)),
            "systems_compared": len(fits), "systems_diverged": diverged,
            "systems_gradient_beyond_fp32_range": beyond,
            f"gtau_last_{window}_steps_along_gpu_trajectory_max": float(max(e_window)),
            f"gtau_last_{window}_steps_along_gpu_trajectory_median": float(np.median(e_window))}, fits


def cpu_baseline_leg(batch, grads, gpu_traj_fn, sample_seconds, threads, avail):
    """The FP64 CPU oracle timed on this host's cores on a bounded sample of
    the same workload (whole systems, the full horizon, forward + adjoint).
    The same sampled systems give the gradient error of the GPU result:
    against the oracle's adjoint along the GPU's own trajectory (the states
    the GPU stepped through, used as the per-step checkpoints), and end to
    end against the oracle's FP64 rollout (dominated by chaotic divergence
    on long horizons)."""
    import oracle as O

    qo, vo, uo = batch.offsets()
    gq0, gqd0, gtau, gparam, gframe = grads
    lo = np.cumsum([0] + [s.n for s in batch.systems])
    n = len(batch.systems)

    def one(i):
        m = O.Model(batch.systems[i], batch.gravity)
        q0, qd0 = batch.q0[qo[i]:qo[i + 1]], batch.qd0[vo[i]:vo[i + 1]]
        tau = np.asarray(batch.tau[:, uo[i]:uo[i + 1]], dtype=np.float64)
        t0 = time.perf_counter()
        qT, qdT = O.rollout(m, q0, qd0, tau, batch.dt)
        r = O.rollout_grad(m, q0, qd0, tau, batch.dt, 2 * qT, np.zeros_like(qdT), K=1)
        return r, time.perf_counter() - t0

    # calibrate on one system, then size the sample to ~sample_seconds of wall time; the second
    # single-threaded run of system 0 gives the single-core figure
    with O.use_library(O.build_native()):
        _, t1 = one(0)
        _, t1 = one(0)
        single_core = batch.systems[0].nv * batch.T / t1
        per_round = max(t1, 1e-3)
        n_sample = int(max(threads, min(n, threads * max(1, int(sample_seconds / per_round)))))
        rng = np.random.default_rng(0)
        idx = sorted(set([0, n - 1] + list(rng.choice(n, size=n_sample, replace=False))))[:n_sample]
        t0 = time.perf_counter()
        res = O.map_threads(one, idx, threads=threads)
        wall = time.perf_counter() - t0
    progress(f"CPU baseline timed: {len(idx)} systems in {wall:.1f} s")
    dof_steps = sum(batch.systems[i].nv for i in idx) * batch.T

    def rel(a, b):
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-6))

    e2e = []
    for (r, _), i in zip(res, idx):
        r0 = O.ball_tangent(batch.systems[i], batch.q0[qo[i]:qo[i + 1]], r[0])
        e = max(rel(gq0[qo[i]:qo[i + 1]], r0), rel(gqd0[vo[i]:vo[i + 1]], r[1]), rel(gtau[:, uo[i]:uo[i + 1]], r[2]))
        if np.isfinite(e):
            e2e.append(e)
    e2e = e2e or [float("nan")]
    # adjoint along the GPU trajectory (not part of the timed baseline)
    trajs = gpu_traj_fn(idx)
    progress("GPU trajectories of the sampled systems copied")
    window = min(batch.T, 2000)
    both = along_errors(batch, grads, idx, trajs, threads, window)
    progress("gradient errors along the GPU trajectory done")
    summ, fits = summarise_along(both, window)
    e_param = [r[1] for r in fits] or [float("nan")]
    cpu = host_cpu()
    base = {"value": dof_steps / wall, "unit": "DOF-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(idx)} of {n} systems, full {batch.T}-step forward+adjoint each "
                      f"(plain dense FP64 C oracle built -O3 -march=native on this host, K=1), {wall:.1f} s wall "
                      f"on {threads} threads of {avail} available, host CPU: {cpu}",
            "host_cpu": cpu, "nproc": os.cpu_count(), "cores_available": avail,
            "single_core_value": single_core,
            "single_core_sample": f"system 0 ({batch.systems[0].nv} DOF), full {batch.T}-step forward+adjoint, "
                                  f"one thread, {t1:.2f} s"}
    err = dict(summ)
    err.update({"end_to_end_vs_fp64_max": max(e2e), "end_to_end_vs_fp64_median": float(np.median(e2e)),
                "param_grads_along_gpu_trajectory_max": max(e_param),
                "param_grads_what": "max over the inertial-parameter and the placement/axis gradients",
                "param_grads_along_gpu_trajectory_median": float(np.median(e_param)),
                "systems": len(idx), "norm": "per system ||g - g_ref|| / ||g_ref||, max over (gq0, gqd0, gtau); "
                                             "elementwise: max |gtau - ref| / max |ref| per system",
                "note": "end-to-end differences on long horizons come from chaotic divergence of FP32 and FP64 "
                        "trajectories; along the GPU's own trajectory what remains is the rounding of the FP32 "
                        "tape (the reverse passes run in FP64 unless adjoint_dtype says f32).  Systems whose "
                        "rollout diverged under the integrator (the FP64 oracle's diverge alike) and systems whose "
                        "exact gradient (FP64, along the GPU trajectory) exceeds the FP32 range are counted, not "
                        "compared: the adjoint of a chaotic rollout grows exponentially backward in time.  The "
                        "last-window figure compares the control gradient over the final steps, which every finite "
                        "system can represent"})
    return base, err, idx, trajs


def memory_sweep(args, torch, dev, sim, b):
    """Forward+adjoint time and peak device memory for checkpoint intervals
    K = 1, 10, 100, store-all and binomial checkpointing with 64 and 16
    snapshots (App. B ablation; Sec. 6 memory tables)."""
    T, dt = b.T, b.dt
    f32 = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device=dev)
    q0, qd0 = f32(b.q0), f32(b.qd0)
    tau = torch.from_numpy(b.tau).to(dev)
    rows = []
    for K in (1, 10, 100, 0, -64, -16):
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        need = sim.workspace_bytes(T, K)
        row = {"K": K if K > 0 else ("store-all" if K == 0 else f"binomial, {-K} snapshots"), "workspace_bytes": need}
        if args.tiling == "auto":
            row["autotune"] = sim.autotune(K=K, T_probe=min(T, 200))
        row["tiling"] = sim.tiling
        try:
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        except RuntimeError as e:
            row["result"] = f"does not fit on the device ({need / 2**30:.1f} GiB workspace): {str(e)[:80]}"
            rows.append(row)
            continue
        times = []
        for rep in range(1 + args.steps):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record()
            qT, qdT, _ = sim.forward(q0, qd0, tau, dt, K=K, workspace=ws)
            e1.record()
            g = sim.backward(tau, dt, K, ws, 2 * qT, torch.zeros_like(qdT))
            e2.record()
            torch.cuda.synchronize()
            if rep:
                times.append((e0.elapsed_time(e1), e1.elapsed_time(e2)))
            del g
        fwd_ms = float(np.mean([t[0] for t in times]))
        bwd_ms = float(np.mean([t[1] for t in times]))
        row.update({"fwd_ms": fwd_ms, "bwd_ms": bwd_ms, "bwd_ms_per_step": bwd_ms / T,
                    "dof_steps_per_s": b.total_dof * T / ((fwd_ms + bwd_ms) * 1e-3),
                    "peak_bytes_over_inputs": int(torch.cuda.max_memory_allocated() - base),
                    "inputs_bytes": int(base)})
        rows.append(row)
        del ws
    print(json.dumps({"metric": "fwd+adjoint DOF-steps/sec and peak memory vs checkpoint interval",
                      "config": {"workload": WORKLOADS.get(b.name, b.name), "T": T, "dt": dt,
                                 "systems": len(b.systems), "dof": b.total_dof},
                      "dtype": "f32", "data": "synthetic", "sweep": rows}))


def rl_bench(args, torch, dev):
    """One-step derivatives for RL (Sec. 5): N samples of one quadruped
    (free base + 12 revolute joints) at random states.  Times, per batch of
    samples, the plain step, the one-step Jacobian-vector product along a
    random action perturbation (sample enhancement: s' + ds'/da . da) and
    the one-step vector-Jacobian product (policy enhancement:
    dQ/ds' . ds'/da), each as one graph replay; checks 16 random samples
    against the FP64 oracle (complex step for the JVP, the adjoint for the
    VJP)."""
    import oracle as O
    from paper_2109_07719_amd import synth
    from paper_2109_07719_amd.sim import Sim

    n = args.rl
    s, _, _, _ = synth.quadruped_system(3000, 1)
    s = synth.round_to_f32(synth.make_batch([(s, np.zeros(s.nq), np.zeros(s.nv), np.zeros((1, s.nu)))], 1e-3)).systems[0]
    rng = np.random.default_rng(17)
    r32 = lambda x: x.astype(np.float32).astype(np.float64)
    q = np.zeros((n, s.nq))
    q[:, :3] = rng.normal(0, 0.2, (n, 3)) + [0, 0.5, 0]
    qt = rng.normal(size=(n, 4))
    q[:, 3:7] = qt / np.linalg.norm(qt, axis=1, keepdims=True)
    q[:, 7:] = rng.normal(0, 0.3, (n, s.nq - 7))
    q = r32(q)
    qd, tau, dtau = r32(rng.normal(0, 0.5, (n, s.nv))), r32(rng.normal(0, 1, (n, s.nu))), r32(rng.normal(0, 1, (n, s.nu)))
    wq, wqd = r32(rng.normal(size=(n, s.nq))), r32(rng.normal(size=(n, s.nv)))
    t0 = time.perf_counter()
    sim = Sim([s] * n, synth.GRAVITY, dtype=torch.float32)
    t_create = time.perf_counter() - t0
    tune = sim.autotune(K=1, T_probe=1) if args.tiling == "auto" else None
    f = lambda x: torch.tensor(np.ascontiguousarray(x).reshape(-1), dtype=torch.float32, device=dev)
    Q, QD, TAU, DTAU, WQ, WQD = f(q), f(qd), f(tau).reshape(1, -1), f(dtau).reshape(1, -1), f(wq), f(wqd)
    Z0, Z1 = torch.zeros_like(Q), torch.zeros_like(QD)
    dt = 1e-3
    ws = sim.new_workspace(1, 1)
    outs = {}

    def plain():
        outs["plain"] = sim.forward(Q, QD, TAU, dt, workspace=None)

    def jvp():
        outs["jvp"] = sim.forward_jvp(Q, QD, TAU, Z0, Z1, DTAU, dt)

    def vjp():
        sim.forward(Q, QD, TAU, dt, K=1, workspace=ws)
        outs["vjp"] = sim.backward(TAU, dt, 1, ws, WQ, WQD)

    fns = {"plain": plain, "jvp": jvp, "vjp": vjp}
    for fn in fns.values():
        fn()
    torch.cuda.synchronize()
    graphs = {}
    for k, fn in fns.items():
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        graphs[k] = g
    res = {}
    for k, g in graphs.items():
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for a, b_ in evs:
            a.record()
            g.replay()
            b_.record()
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b_) for a, b_ in evs]))
        res[k] = {"ms_per_batch": ms, "samples_per_s": n / (ms * 1e-3)}
    # FP64 oracle checks on 16 samples
    m = O.Model(s, synth.GRAVITY)
    (_, _, dqT, dqdT) = [x.cpu().numpy().reshape(n, -1) for x in outs["jvp"]]
    gq0, gqd0, gtau = [x.cpu().numpy().reshape(n, -1) for x in outs["vjp"]]
    ej, ev = [], []
    h = 1e-30
    for i in rng.choice(n, 16, replace=False):
        cq, cqd = O.rollout_complex(m, q[i].astype(complex), qd[i].astype(complex), (tau[i] + 1j * h * dtau[i])[None], dt)
        ej.append(max(_rel(dqT[i], cq.imag / h), _rel(dqdT[i], cqd.imag / h)))
        g = O.rollout_grad(m, q[i], qd[i], tau[i][None], dt, wq[i], wqd[i])
        ev.append(max(_rel(gq0[i], g[0]), _rel(gqd0[i], g[1]), _rel(gtau[i], g[2][0])))
    print(json.dumps({"metric": "one-step derivative samples/s (FP32, 1 GPU) for RL sample and policy enhancement",
                      "config": {"workload": f"{n} samples of one free-floating quadruped (base + 4x3 revolute, "
                                             "13 bodies, n_q=19, n_v=18) at random states, one step dt=1e-3",
                                 "samples": n, "tiling": sim.tiling, "autotune": tune, "create_s": t_create},
                      "dtype": "f32", "data": "synthetic", "results": res,
                      "fp64_oracle_rel_err_16_samples": {"jvp_max": max(ej), "vjp_max": max(ev)},
                      "nonfinite_outputs": sim.status()}))


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-6))


def _rel_floor(a, b, floor):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), floor))


def contact_bench(args, torch, dev):
    """Rollouts with contact inside the step and their gradient (Sec. 4.1
    "Collision resolution"): B landing quadrupeds (spheres on the four feet),
    T steps, one launch each way, timed with HIP events on the launch stream.
    FLOPs per step are counted by the library at sampled states of the
    timed trajectory; the FP64 oracle (step with contact and its complex-step
    gradient) is timed on the host on whole systems over a short window."""
    import ctypes

    import oracle as O
    from paper_2109_07719_amd import _native as N
    from paper_2109_07719_amd import synth
    from paper_2109_07719_amd.contact import ContactBatch, pack_params

    B, T = (int(v) for v in args.contact.split(","))
    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    mu, beta, niter, dt, G = 0.8, 0.2, 30, 1e-3, (0.0, -9.81, 0.0)
    draws = [synth.landing_quadruped(50000 + i, T) for i in range(B)]
    cb = ContactBatch([d[0] for d in draws], draws[0][4], [d[5] for d in draws], [d[6] for d in draws], mu=mu,
                      beta=beta, niter=niter, gravity=G, dtype=dtype)
    f = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=dev)
    q0 = f(np.stack([d[1] for d in draws], axis=1))
    qd0 = f(np.stack([d[2] for d in draws], axis=1))
    tau = f(np.stack([d[3] for d in draws], axis=2))
    gqT = torch.ones_like(q0)
    gqdT = torch.ones_like(qd0)
    # launch geometry (systems per wave of both kernels), tuned on 50 probe
    # steps from the middle of an untimed rollout, where the feet are on the
    # ground (the first ~30 steps are free fall, much cheaper per step)
    tune = None
    if args.tiling == "auto" and T > 0:
        _, _, tr = cb.rollout(q0, qd0, tau, dt)
        t0 = T // 2
        x0 = tr[t0].contiguous()
        tune = cb.autotune(x0[:cb.nq].contiguous(), x0[cb.nq:].contiguous(), tau[t0:t0 + 50].contiguous(), dt)
        tune["probe"] = f"steps {t0}..{min(T, t0 + 50)} of an untimed rollout"
        del tr
    for _ in range(max(args.warmup, 1)):
        qT, qdT, tr, nc = cb.rollout(q0, qd0, tau, dt, counts=True)
        g = cb.grad(tr, tau, dt, gqT, gqdT)
    torch.cuda.synchronize()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    fwd_ms, grad_ms = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e0, e1, e2 = ev(), ev(), ev()
        e0.record()
        qT, qdT, tr, nc = cb.rollout(q0, qd0, tau, dt, counts=True)
        e1.record()
        g = cb.grad(tr, tau, dt, gqT, gqdT)
        e2.record()
        torch.cuda.synchronize()
        fwd_ms.append(e0.elapsed_time(e1))
        grad_ms.append(e1.elapsed_time(e2))
        print(f"contact step: rollout {fwd_ms[-1]:.2f} ms, gradient {grad_ms[-1]:.2f} ms", file=sys.stderr, flush=True)
    wall = (time.perf_counter() - t0) / args.steps
    fwd, grd = float(np.mean(fwd_ms)), float(np.mean(grad_ms))
    ncn = nc.cpu().numpy()
    # FLOPs at sampled (system, step) states of the timed trajectory
    rng = np.random.default_rng(3)
    trn = tr.double().cpu().numpy()
    taun = tau.double().cpu().numpy()
    par, jt = (np.ascontiguousarray(x, np.int32) for x in (draws[0][0].parent, draws[0][0].jtype))
    sf, gf = [], []
    for _ in range(48):
        i, t = int(rng.integers(B)), int(rng.integers(T))
        P = np.ascontiguousarray(pack_params(draws[i][0], draws[i][5], draws[i][6]))
        x = np.ascontiguousarray(trn[t, :, i])
        u = np.ascontiguousarray(taun[t, :, i])
        a, b = ctypes.c_double(), ctypes.c_double()
        N.check(N.lib().sim_contact_flops(ctypes.byref(cb.m), P.ctypes.data, x.ctypes.data,
                                          x[cb.nq:].ctypes.data, u.ctypes.data, dt, ctypes.byref(a), ctypes.byref(b)))
        sf.append(a.value)
        gf.append(b.value)
    fl_fwd, fl_grad = float(np.mean(sf)) * B * T, float(np.mean(gf)) * B * T
    # parity sample: the GPU's steps from its own states against the oracle's
    worst = 0.0
    for i in range(0, B, max(1, B // 8)):
        m = O.Model(draws[i][0], G)
        C = O.Contacts(draws[i][4], draws[i][5], draws[i][6], mu=mu, beta=beta, niter=niter)
        for t in range(0, T, max(1, T // 10)):
            x = trn[t, :, i]
            q1, qd1, _, _ = O.step_contact(m, C, x[:cb.nq], x[cb.nq:], taun[t, :, i], dt)
            worst = max(worst, _rel(trn[t + 1, :, i], np.r_[q1, qd1]))
    # the FP32 gradient of the whole rollout against the oracle's one-step
    # gradients chained backwards along the GPU's own trajectory, on sampled
    # systems, with the model as the GPU holds it (rounded to FP32)
    r32 = lambda x: np.asarray(x, dtype=np.float32).astype(np.float64)
    gn = [x.double().cpu().numpy() for x in g[:3]]
    sample = list(range(0, B, max(1, B // 8)))
    dt32 = float(r32(dt))

    def along(i):
        s = draws[i][0]
        s32 = synth.System(parent=s.parent, jtype=s.jtype, E_T=r32(s.E_T), r_T=r32(s.r_T), axis=r32(s.axis),
                           mass=r32(s.mass), com=r32(s.com), Ic=r32(s.Ic))
        m = O.Model(s32, r32(G))
        C = O.Contacts(draws[i][4], r32(draws[i][5]), r32(draws[i][6]), mu=float(r32(mu)), beta=float(r32(beta)),
                       niter=niter)
        gq, gqd = np.ones(cb.nq), np.ones(cb.nv)
        gt = np.zeros((T, cb.nu))
        for t in range(T - 1, -1, -1):
            x = trn[t, :, i]
            gq, gqd, gtt = O.rollout_contact_grad(m, C, x[:cb.nq], x[cb.nq:], taun[t:t + 1, :, i], dt32, gq, gqd)
            gt[t] = gtt[0]
        got = (gn[0][:, i], gn[1][:, i], gn[2][:, :, i])
        scale = max(float(np.abs(r).max()) for r in (gq, gqd, gt))
        return max(_rel_floor(a, b, 1e-6 * scale) for a, b in zip(got, (gq, gqd, gt)))

    grad_err = O.map_threads(along, sample, threads=host_threads()[0])
    progress(f"contact gradient along the GPU trajectory on {len(sample)} systems: max {max(grad_err):.2e}")
    cpu = None
    if not args.no_cpu_baseline:
        Tw = min(T, 40)
        t0, dof_steps, k = time.perf_counter(), 0, 0
        while time.perf_counter() - t0 < min(args.cpu_sample_seconds, 15.0):
            d = draws[k % B]
            m = O.Model(d[0], G)
            C = O.Contacts(d[4], d[5], d[6], mu=mu, beta=beta, niter=niter)
            O.rollout_contact(m, C, d[1], d[2], d[3][:Tw], dt)
            O.rollout_contact_grad(m, C, d[1], d[2], d[3][:Tw], dt, np.ones(cb.nq), np.ones(cb.nv))
            dof_steps += cb.nv * Tw
            k += 1
        cpu = {"value": dof_steps / (time.perf_counter() - t0), "unit": "DOF-steps/s", "cores": 1, "kind": "oracle",
               "sample": f"{k} whole quadrupeds x {Tw} steps (fall and touchdown), FP64 step with contact + "
                         f"complex-step gradient, one host thread"}
    total = fwd + grd
    res = {"metric": "contact rollout forward+gradient DOF-steps/s (1 GPU)", "value": B * cb.nv * T / (total * 1e-3),
           "unit": "DOF-steps/s", "higher_is_better": True, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": total, "wall_ms_per_step": wall * 1e3, "scaling": "weak",
           "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
           "config": {"workload": f"{B} landing quadrupeds (18 DOF, contact spheres on 4 feet), T={T}, dt=1e-3, "
                                  f"PGS {niter} sweeps x 2 solves, mu {mu}, beta {beta}",
                      "batch": B, "T": T, "tiling": cb.tiling, "autotune": tune},
           "rollout_ms": fwd, "gradient_ms": grd,
           "active_contacts_per_step": {str(k): int(v) for k, v in enumerate(np.bincount(ncn.reshape(-1), minlength=5))},
           # the gradient kernel recomputes and reverses every step in FP64 (both dtypes)
           "roofline": {"bound": "alu", "kernel": "k_contact_adj", "achieved": fl_grad / (grd * 1e-3) / 1e12,
                        "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": fl_grad / (grd * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                        "traffic": None, "flops_per_launch": fl_grad,
                        "rollout_achieved": fl_fwd / (fwd * 1e-3) / 1e12, "rollout_flops_per_launch": fl_fwd,
                        "flops_per_step_mean": float(np.mean(sf)), "grad_flops_per_step_mean": float(np.mean(gf))},
           "step_map_error_vs_oracle_max": worst,
           "grad_rel_err": {"along_gpu_trajectory_max": max(grad_err),
                            "along_gpu_trajectory_median": float(np.median(grad_err)), "systems": len(sample),
                            "what": "per system max over (q0_bar, qd0_bar, tau_bar) of ||g - ref|| / ||ref|| "
                                    "(floor 1e-6 x the largest entry), ref = the FP64 oracle's one-step gradients "
                                    "chained backwards along the GPU's own FP32 trajectory over all T steps; "
                                    "bar 1e-3 (FP32 gradients)"},
           "cpu_baseline": cpu}
    print(json.dumps(res))


def pgs_bench(args, torch, dev):
    """Contact solver (Sec. 4.1 "Collision resolution", Eq. mlcp; App. C):
    a batch of independent MLCPs a = A x + b, lo <= x <= hi solved by a fixed
    number of projected Gauss-Seidel sweeps, and the adjoint sweep.  Inputs:
    Delassus-like A = Q diag(1..8) Q^T plus a small non-symmetric part,
    b ~ N(0, 1.5^2), box half-widths U(0.05, 0.6) (30 % of rows one-sided,
    lo = 0), x0 ~ N(0, 0.3^2), FP32.  Times the solve (keeping the sweep
    vectors) and the adjoint as graph replays with HIP events; checks 64
    problems against the FP64 oracle; times the oracle on the host."""
    import oracle as O
    from paper_2109_07719_amd import pgs

    B, n, niter = (int(v) for v in args.pgs.split(","))
    rng = np.random.default_rng(21)
    nb = min(B, 1024)   # distinct problems, tiled through the batch
    A = np.empty((nb, n, n))
    for p in range(nb):
        Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
        A[p] = Q @ np.diag(np.linspace(1.0, 8.0, n)) @ Q.T + 0.2 * rng.normal(size=(n, n))
        A[p][np.diag_indices(n)] = np.abs(A[p][np.diag_indices(n)]) + 1.0
    half = rng.uniform(0.05, 0.6, (nb, n))
    lo, hi = -half, half.copy()
    one = rng.uniform(size=(nb, n)) < 0.3
    lo[one], hi[one] = 0.0, 3e38
    b, x0 = rng.normal(0, 1.5, (nb, n)), rng.normal(0, 0.3, (nb, n))
    idx = np.arange(B) % nb
    r32 = lambda x: x.astype(np.float32).astype(np.float64)
    A, b, lo, hi, x0 = (r32(v[idx]) for v in (A, b, lo, hi, x0))
    xbar = r32(rng.normal(size=(B, n)))
    f = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device=dev)
    tA, tb, tlo, thi, tx0, txb = f(A), f(b), f(lo), f(hi), f(x0), f(xbar)
    ws = pgs.new_workspace(B, n, niter)
    x = torch.empty_like(tb)
    gout = tuple(torch.empty_like(t) for t in (tA, tb, tb, tb, tb))
    solve = lambda: pgs.solve(tA, tb, tlo, thi, tx0, niter, workspace=ws, out=x)
    adj = lambda: pgs.adjoint(tA, tb, tlo, thi, txb, niter, ws, out=gout)
    solve(), adj()
    torch.cuda.synchronize()
    graphs = {}
    for k, fn in (("solve", solve), ("adjoint", adj)):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        graphs[k] = g
    ms = {}
    for k, g in graphs.items():
        for _ in range(max(args.warmup, 2)):
            g.replay()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for e0, e1 in evs:
            e0.record()
            g.replay()
            e1.record()
        torch.cuda.synchronize()
        ms[k] = float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))
    # algorithmic work per problem (FP32): a row update is the (n-1)-term
    # dot product, the add of b and the division; the adjoint row recomputes
    # it and adds the b, A and x adjoints
    fl_solve = niter * n * (2 * (n - 1) + 2)
    fl_adj = niter * n * (6 * (n - 1) + 7)
    by_solve = 4 * (n * n + 4 * n + n + (niter + 1) * n)
    by_adj = 4 * (n * n + 4 * n + 2 * niter * n + n * n + 4 * n)
    gx, gg = x.cpu().numpy(), [t.cpu().numpy() for t in gout]
    errs = []
    for p in rng.choice(B, 64, replace=False):
        xr, sw = O.pgs_solve(A[p], b[p], lo[p], hi[p], x0[p], niter, sweeps=True)
        gr = O.pgs_adjoint(A[p], b[p], lo[p], hi[p], sw, xbar[p])
        errs.append(max(_rel(gx[p], xr), max(_rel(gg[k][p], gr[k]) for k in range(5))))
    # the FP64 oracle on the host, one thread, solve + adjoint per problem
    t0, k = time.perf_counter(), 0
    while time.perf_counter() - t0 < min(args.cpu_sample_seconds, 5.0):
        p = k % nb
        xr, sw = O.pgs_solve(A[p], b[p], lo[p], hi[p], x0[p], niter, sweeps=True)
        O.pgs_adjoint(A[p], b[p], lo[p], hi[p], sw, xbar[p])
        k += 1
    cpu_rate = k / (time.perf_counter() - t0)
    total = ms["solve"] + ms["adjoint"]
    res = {"metric": "MLCP solve+adjoint problems/s (projected Gauss-Seidel, FP32, 1 GPU)",
           "value": B / (total * 1e-3), "unit": "problems/s", "higher_is_better": True,
           "ms_per_step": total, "steps": args.steps, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{B} MLCPs of {n} rows (Delassus-like A, box and one-sided bounds), "
                                  f"{niter} sweeps, solve keeping the sweep vectors + adjoint",
                      "batch": B, "rows": n, "sweeps": niter, "lanes_per_problem": 1},
           "solve_ms": ms["solve"], "adjoint_ms": ms["adjoint"],
           "roofline": {"bound": "alu", "unit": "TFLOP/s", "peak": FP32_PEAK_TFLOPS,
                        "solve_achieved": fl_solve * B / (ms["solve"] * 1e-3) / 1e12,
                        "adjoint_achieved": fl_adj * B / (ms["adjoint"] * 1e-3) / 1e12,
                        "solve_hbm_gb_per_s": by_solve * B / (ms["solve"] * 1e-3) / 1e9,
                        "adjoint_hbm_gb_per_s": by_adj * B / (ms["adjoint"] * 1e-3) / 1e9,
                        "flops_per_problem": {"solve": fl_solve, "adjoint": fl_adj},
                        "bytes_per_problem": {"solve": by_solve, "adjoint": by_adj}},
           "fp64_oracle_rel_err_64_problems": {"max": max(errs), "median": float(np.median(errs))},
           "cpu_baseline": {"value": cpu_rate, "unit": "problems/s", "cores": 1, "kind": "oracle",
                            "sample": f"{k} problems, FP64 C oracle solve + adjoint, one thread"}}
    res["roofline"]["frac"] = res["roofline"]["adjoint_achieved"] / FP32_PEAK_TFLOPS
    print(json.dumps(res))


def fp64_leg(args, torch, dev, b, K, T, dt):
    """The same rollouts with the FP64 handle (context for accuracy-critical
    uses; not the headline): forward with checkpoints and adjoint, timed with
    HIP events like the FP32 legs.  Skipped when the workspace would not
    fit."""
    from paper_2109_07719_amd.sim import Sim
    sim = Sim(b.systems, b.gravity, dtype=torch.float64)
    need = sim.workspace_bytes(T, K)
    if K < 1 or need > 0.5 * torch.cuda.mem_get_info()[0]:
        return {"skipped": f"needs {need / 2**30:.1f} GiB of workspace (K={K})"}
    tune = sim.autotune(K=K, T_probe=min(T, 200)) if args.tiling == "auto" else None
    f = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)
    q0, qd0 = f(b.q0), f(b.qd0)
    tau = torch.from_numpy(b.tau).to(dev).double()
    ws = sim.new_workspace(T, K)
    times = []
    for k in range(args.warmup + args.steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        qT, qdT, _ = sim.forward(q0, qd0, tau, dt, K=K, workspace=ws)
        e[1].record()
        sim.backward(tau, dt, K, ws, 2 * qT, torch.zeros_like(qdT))
        e[2].record()
        torch.cuda.synchronize()
        if k >= args.warmup:
            times.append((e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])))
    fw, bw = float(np.mean([t[0] for t in times])), float(np.mean([t[1] for t in times]))
    del ws, tau
    return {"fwd_adjoint_dof_steps_per_s": b.total_dof * T / ((fw + bw) * 1e-3), "fwd_kernel_ms": fw,
            "adjoint_kernel_ms": bw, "tiling": sim.tiling, "autotune": tune,
            "what": "the same rollouts in FP64 (the library's FP64 handle): the price of full accuracy, where the "
                    "FP32 gradients of long or chaotic rollouts lose digits; not the headline value"}


def trajopt_bench(args, torch, dev):
    """Trajectory optimisation: 2048 chains of 5-50 links, T=1000, Adam on
    tau; reports DOF-steps/s per iteration (forward+adjoint of every chain),
    the loss curve and FP64 oracle gradient spot-checks."""
    from paper_2109_07719_amd.trajopt import TrajOpt, chains_problem

    T = args.T or 1000
    b, targets = chains_problem(n_systems=2048, T=T)
    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    opt = TrajOpt(b, targets, [s.n - 1 for s in b.systems], np.tile([0.5, 0, 0], (2048, 1)), K=args.K,
                  dtype=dtype)
    tune = opt.sim.autotune(K=args.K, T_probe=min(T, 200)) if args.tiling == "auto" else None
    checks = {0, args.trajopt // 2, args.trajopt - 1}
    losses, it_ms, spot = [], [], []
    for it in range(args.trajopt):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        opt.opt.zero_grad()
        L, _ = opt.loss()
        L.backward()
        e1.record()
        torch.cuda.synchronize()
        it_ms.append(e0.elapsed_time(e1))
        losses.append(float(L.detach()))
        if it in checks and not args.no_cpu_baseline:
            spot.append({"iteration": it, **_trajopt_spot_check(opt, b, targets, torch)})
        opt.opt.step()
    torch.cuda.synchronize()
    ms = float(np.mean(it_ms[1:] if len(it_ms) > 1 else it_ms))
    print(json.dumps({"metric": f"fwd+adjoint DOF-steps/sec ({args.dtype.upper()}, 1 GPU) in trajectory optimisation",
                      "value": b.total_dof * T / (ms * 1e-3), "unit": "DOF-steps/s", "ms_per_iteration": ms,
                      "iterations": args.trajopt, "loss_first": losses[0], "loss_last": losses[-1],
                      "loss_every_10": losses[::10], "fp64_spot_checks": spot, "dtype": args.dtype,
                      "config": {"workload": WORKLOADS["chains_2048"], "systems": 2048, "dof": b.total_dof,
                                 "T": T, "K": args.K, "tiling": opt.sim.tiling, "autotune": tune}}))


def _trajopt_spot_check(opt, b, targets, torch):
    """dL/dtau of 16 random chains against the FP64 oracle: (a) along the
    GPU's own trajectory (its states as per-step checkpoints, seed from torch
    FP64 forward kinematics at the GPU's q^T), (b) end to end (the oracle's
    own FP64 rollout; long chains falling under gravity are chaotic, so (b)
    includes trajectory divergence)."""
    import oracle as O
    from paper_2109_07719_amd.fk import LinkPoints
    qo, vo, uo = b.offsets()
    tau_dev = opt.tau.detach()
    tau = tau_dev.double().cpu().numpy()
    g = opt.tau.grad.detach().cpu().numpy()
    _, _, tr = opt.sim.forward(opt.q0, opt.qd0, tau_dev, b.dt, K=1, workspace=None, traj=True)
    nq = opt.sim.nq
    rng = np.random.default_rng(1)
    along, e2e = 0.0, 0.0
    rel = lambda a, r: float(np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-6))
    for i in rng.choice(len(b.systems), size=16, replace=False):
        s = b.systems[i]
        m = O.Model(s, b.gravity)
        ti = tau[:, uo[i]:uo[i + 1]]
        fk = LinkPoints([s], [s.n - 1], [[0.5, 0, 0]], dtype=torch.float64, device="cpu")
        cols = torch.from_numpy(np.r_[qo[i]:qo[i + 1], nq + vo[i]:nq + vo[i + 1]]).to(tr.device)
        traj_i = tr[:, cols].double().cpu().numpy()
        x0 = np.r_[b.q0[qo[i]:qo[i + 1]], b.qd0[vo[i]:vo[i + 1]]]
        states = np.concatenate([x0[None], traj_i[:-1]])

        def seed(qT):
            qt = torch.tensor(qT, requires_grad=True)
            ((fk(qt) - torch.tensor(targets[i:i + 1])) ** 2).sum().backward()
            return qt.grad.numpy()

        ga = O.adjoint_along(m, states, ti, b.dt, seed(traj_i[-1, :s.nq]), np.zeros(s.nv))
        along = max(along, rel(g[:, uo[i]:uo[i + 1]], ga[2] + 2 * opt.w * ti))
        qT, _ = O.rollout(m, x0[:s.nq], x0[s.nq:], ti, b.dt)
        ref = O.rollout_grad(m, x0[:s.nq], x0[s.nq:], ti, b.dt, seed(qT), np.zeros(s.nv))
        e2e = max(e2e, rel(g[:, uo[i]:uo[i + 1]], ref[2] + 2 * opt.w * ti))
    return {"along_gpu_trajectory_max": along, "end_to_end_vs_fp64_max": e2e}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed steps (each = full forward+adjoint rollout)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chain7_4096", choices=sorted(WORKLOADS))
    ap.add_argument("--K", type=int, default=1, help="checkpoint interval")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 context leg")
    ap.add_argument("--no-fp32-adjoint", action="store_true",
                    help="skip the context leg with the adjoint's reverse passes in FP32")
    ap.add_argument("--dtype", choices=("f32", "f64"), default="f32",
                    help="compute type of the trajectory-optimisation leg (the benchmark line is FP32)")
    ap.add_argument("--cpu-sample-seconds", type=float, default=15.0)
    ap.add_argument("--memory-sweep", action="store_true",
                    help="time forward+adjoint and record peak memory for K in 1,10,100 and store-all")
    ap.add_argument("--trajopt", type=int, default=0,
                    help="run this many Adam iterations of trajectory optimisation (chains_2048 workload)")
    ap.add_argument("--rl", type=int, default=0,
                    help="one-step JVP/VJP throughput for RL on this many quadruped samples (Sec. 5)")
    ap.add_argument("--contact", default="", help="B,T: rollouts with contact and their gradient")
    ap.add_argument("--pgs", default="",
                    help="B,n,niter: time the contact solver (MLCP projected Gauss-Seidel) and its adjoint instead")
    ap.add_argument("--T", type=int, default=None, help="override the horizon (reduced runs only)")
    ap.add_argument("--tiling", default="auto",
                    help="launch geometry: 'auto' (the library's autotuner, before the timed region), 'default' "
                         "(occupancy rule), or W,P,PIPE = waves per workgroup, producer/consumer pairs per "
                         "workgroup, pipelined adjoint (1/0)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(systems shard across GPUs with no communication; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": n * 4, "calib_copy_bytes_written": n * 4, "launches": 5}))
        return

    from paper_2109_07719_amd import synth
    from paper_2109_07719_amd.sim import Sim

    if args.trajopt:
        return trajopt_bench(args, torch, dev)
    if args.rl:
        return rl_bench(args, torch, dev)
    if args.pgs:
        return pgs_bench(args, torch, dev)
    if args.contact:
        return contact_bench(args, torch, dev)

    t_gen = time.perf_counter()
    b = synth.workload(args.workload, T=args.T, tau_dtype=np.float32)
    # the oracle and the GPU see the same float32-rounded inputs
    r = synth.round_to_f32(synth.Batch(systems=b.systems, q0=b.q0, qd0=b.qd0, tau=b.tau[:1], dt=b.dt))
    b = synth.Batch(systems=r.systems, q0=r.q0, qd0=r.qd0, tau=b.tau, dt=r.dt, gravity=r.gravity, name=b.name)
    t_gen = time.perf_counter() - t_gen

    sim = Sim(b.systems, b.gravity, dtype=torch.float32)
    tune = None
    if args.tiling == "auto":
        t0 = time.perf_counter()
        tune = sim.autotune(K=args.K, T_probe=min(b.T, 200))
        tune["seconds"] = time.perf_counter() - t0
    elif args.tiling != "default":
        w, p_, pipe = (int(x) for x in args.tiling.split(","))
        sim.set_tiling(w, p_, bool(pipe))
    if args.memory_sweep:
        return memory_sweep(args, torch, dev, sim, b)
    T, K, dt = b.T, args.K, b.dt
    f32 = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device=dev)
    q0, qd0 = f32(b.q0), f32(b.qd0)
    tau = torch.from_numpy(b.tau).to(dev)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base_mem = torch.cuda.memory_allocated()
    ws = sim.new_workspace(T, K)
    qT = torch.empty(sim.nq, dtype=torch.float32, device=dev)
    qdT = torch.empty(sim.nv, dtype=torch.float32, device=dev)
    gqdT = torch.zeros(sim.nv, dtype=torch.float32, device=dev)
    gqT = torch.empty(sim.nq, dtype=torch.float32, device=dev)
    gq0 = torch.empty(sim.nq, dtype=torch.float32, device=dev)
    gqd0 = torch.empty(sim.nv, dtype=torch.float32, device=dev)
    gtau = torch.empty((T, sim.nu), dtype=torch.float32, device=dev)
    pqT = torch.empty_like(qT)
    pqdT = torch.empty_like(qdT)

    def fwd():
        sim.forward(q0, qd0, tau, dt, K=K, workspace=ws, out=(qT, qdT, None))
        torch.mul(qT, 2.0, out=gqT)   # loss L = sum q_T^2

    def bwd():
        sim.backward(tau, dt, K, ws, gqT, gqdT, out=(gq0, gqd0, gtau))

    gparam = torch.empty((sim.info["n_links"], 10), dtype=torch.float32, device=dev)
    gframe = torch.empty((sim.info["n_links"], 9), dtype=torch.float32, device=dev)

    def bwd_params():
        sim.backward(tau, dt, K, ws, gqT, gqdT, out=(gq0, gqd0, gtau, gparam, gframe), params=True)

    def plain():
        sim.forward(q0, qd0, tau, dt, K=K, workspace=None, out=(pqT, pqdT, None))

    # warm up eagerly once (also the first correctness pass), then capture
    fwd(), bwd(), plain(), bwd_params()
    torch.cuda.synchronize()
    def step():
        fwd()
        bwd()

    graphs = {}
    for name, fn in (("step", step), ("fwd", fwd), ("bwd", bwd), ("plain", plain), ("bwd_params", bwd_params)):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        graphs[name] = g
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        graphs["step"].replay()
        graphs["plain"].replay()
    torch.cuda.synchronize()

    # timed region: forward + adjoint as one captured graph, K steps, events
    # on the launch stream
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record()
        graphs["step"].replay()
        ev[k][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [ev[k][0].elapsed_time(ev[k][2]) for k in range(args.steps)]
    peak_mem = torch.cuda.max_memory_allocated() - base_mem
    # per-kernel split (roofline): the forward and the adjoint graphs replayed
    # with an event between them, as many times again
    for k in range(args.steps):
        ev[k][0].record()
        graphs["fwd"].replay()
        ev[k][1].record()
        graphs["bwd"].replay()
        ev[k][2].record()
    torch.cuda.synchronize()
    fwd_ms = [ev[k][0].elapsed_time(ev[k][1]) for k in range(args.steps)]
    bwd_ms = [ev[k][1].elapsed_time(ev[k][2]) for k in range(args.steps)]

    # plain forward (no checkpoints), same timing method
    pev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    for k in range(args.steps):
        pev[k][0].record()
        graphs["plain"].replay()
        pev[k][1].record()
    torch.cuda.synchronize()
    plain_ms = [pev[k][0].elapsed_time(pev[k][1]) for k in range(args.steps)]
    # adjoint with model-parameter gradients (outside the headline value)
    graphs["fwd"].replay()
    for k in range(args.steps):
        pev[k][0].record()
        graphs["bwd_params"].replay()
        pev[k][1].record()
    torch.cuda.synchronize()
    bwd_params_ms = [pev[k][0].elapsed_time(pev[k][1]) for k in range(args.steps)]
    # the same adjoint with its reverse passes in FP32 (context: faster, but
    # it loses digits on long or chaotic rollouts; the headline runs them in
    # FP64 from the FP32 tape)
    adj32 = None
    if not args.no_fp32_adjoint:
        # the launch geometry is tuned for the FP64 reverse passes; the FP32
        # ones get their own tuning (two producer/consumer pairs per
        # workgroup matter there), and the FP64 choice is restored after
        tiling64 = sim.tiling
        sim.set_adjoint_dtype(torch.float32)
        if args.tiling == "auto":
            sim.autotune(K)
        g32 = [torch.empty_like(x) for x in (gq0, gqd0, gtau)]
        graphs["fwd"].replay()
        sim.backward(tau, dt, K, ws, gqT, gqdT, out=tuple(g32))
        torch.cuda.synchronize()
        gb32 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gb32):
            sim.backward(tau, dt, K, ws, gqT, gqdT, out=tuple(g32))
        for k in range(args.steps):
            pev[k][0].record()
            gb32.replay()
            pev[k][1].record()
        torch.cuda.synchronize()
        b32_ms = float(np.mean([pev[k][0].elapsed_time(pev[k][1]) for k in range(args.steps)]))
        adj32 = {"kernel_ms": b32_ms,
                 "fwd_adjoint_dof_steps_per_s": b.total_dof * T / ((float(np.mean(fwd_ms)) + b32_ms) * 1e-3),
                 "achieved_tflops": sim.flops(2) * T / (b32_ms * 1e-3) / 1e12,
                 "tiling": sim.tiling, "grads": [x.cpu().numpy() for x in g32]}
        sim.set_adjoint_dtype(torch.float64)
        sim.set_tiling(**tiling64)
        del gb32
    # leave the graphs' gradient buffers as the plain adjoint wrote them
    graphs["bwd"].replay()
    torch.cuda.synchronize()

    progress(f"timed legs done: forward+adjoint {float(np.mean(step_ms)):.2f} ms per step")
    fp64 = None if args.no_fp64 else fp64_leg(args, torch, dev, b, K, T, dt)
    progress("FP64 context leg done")

    grads = (gq0.cpu().numpy(), gqd0.cpu().numpy(), gtau.cpu().numpy(), gparam.cpu().numpy(), gframe.cpu().numpy())
    finite = all(np.all(np.isfinite(g)) for g in grads) and bool(torch.isfinite(qT).all())
    nonfinite_outputs = sim.status()
    dof_steps = b.total_dof * T
    ms_per_step = float(np.mean(step_ms))
    value = dof_steps / (ms_per_step * 1e-3)
    plain_rate = dof_steps / (float(np.mean(plain_ms)) * 1e-3)

    bwd_flops = sim.flops(2) * T
    fwd_flops = sim.flops(1) * T
    bwd_s = float(np.mean(bwd_ms)) * 1e-3
    achieved = bwd_flops / bwd_s / 1e12
    bwd_kernel = "k_backward_pipe" if (K == 1 and sim.tiling["pipelined"]) else "k_backward"
    # the adjoint kernel's arithmetic is FP64 (recompute and reverse passes)
    # unless the FP32 backward was selected
    adj64 = sim.adjoint_dtype == torch.float64
    peak = FP64_PEAK_TFLOPS if adj64 else FP32_PEAK_TFLOPS
    roofline = {"bound": "alu", "kernel": bwd_kernel, "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak,
                "peak_what": ("MI355X FP64 vector peak (the adjoint kernel computes in FP64)" if adj64 else
                              "MI355X FP32 vector peak"),
                "frac_of_fp32_peak": achieved / FP32_PEAK_TFLOPS,
                "traffic": traffic_entry(bwd_kernel, args.workload),
                "flops_per_launch": bwd_flops, "kernel_ms": float(np.mean(bwd_ms)),
                "fwd_kernel_ms": float(np.mean(fwd_ms)),
                "fwd_achieved_tflops": fwd_flops / (float(np.mean(fwd_ms)) * 1e-3) / 1e12,
                "kernel_ms_median": float(np.median(bwd_ms)), "fwd_kernel_ms_median": float(np.median(fwd_ms))}
    if roofline["traffic"] is not None:
        roofline["hbm_gb_per_s"] = roofline["traffic"] / bwd_s / 1e9

    out = {"metric": "fwd+adjoint DOF-steps/sec (FP32, 1 GPU) vs plain fwd; grad rel err",
           "value": value, "unit": "DOF-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_per_step, "ms_per_step_median": float(np.median(step_ms)), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "adjoint_dtype": "f64" if sim.adjoint_dtype == torch.float64 else "f32",
           "precision": "FP32 inputs, outputs, checkpoints and forward rollout; the backward pass recomputes each "
                        "step from its widened FP32 checkpoint and runs the reverse passes and the adjoint state "
                        "carried between steps in FP64, rounding its outputs to FP32 once",
           "data": "synthetic",
           "config": {"workload": WORKLOADS[args.workload], "systems": len(b.systems), "dof": b.total_dof,
                      "T": T, "dt": dt, "K": K, "lanes": sim.info["n_slots"], "waves": sim.info["n_waves"],
                      "lanes_per_system": "one lane per link", "tiling": sim.tiling,
                      "autotune": tune, "timed": "one HIP graph replay per step holding the forward and the adjoint"},
           "plain_fwd_dof_steps_per_s": plain_rate,
           "adjoint_with_param_grads": {"kernel_ms": float(np.mean(bwd_params_ms)),
                                        "fwd_adjoint_dof_steps_per_s":
                                            dof_steps / ((float(np.mean(fwd_ms)) + float(np.mean(bwd_params_ms))) * 1e-3),
                                        "what": "gradients with respect to every link's 10 inertial parameters "
                                                "and its joint placement and axis (9) as well, summed over the "
                                                "rollout"}, "fwd_adjoint_over_plain_fwd_time": value and plain_rate / value,
           "fp64_handle": fp64,
           "peak_mem_bytes": int(peak_mem), "results_finite": finite, "nonfinite_outputs": nonfinite_outputs, "roofline": roofline,
           "wall_s_timed": wall, "input_gen_s": t_gen}
    if not args.no_cpu_baseline:
        threads, avail = host_threads()
        traj_dev = torch.empty((T, sim.nq + sim.nv), dtype=torch.float32, device=dev)
        sim.forward(q0, qd0, tau, dt, K=K, workspace=None, traj=True, out=(pqT, pqdT, traj_dev))
        torch.cuda.synchronize()
        qo, vo, _ = b.offsets()

        def gpu_traj(idx):
            out_ = []
            for i in idx:
                cols = np.r_[qo[i]:qo[i + 1], sim.nq + vo[i]:sim.nq + vo[i + 1]]
                out_.append(traj_dev[:, torch.from_numpy(cols).to(dev)].double().cpu().numpy())
            return out_

        base, err, idx, trajs = cpu_baseline_leg(b, grads, gpu_traj, args.cpu_sample_seconds, threads, avail)
        del traj_dev
        out["cpu_baseline"] = base
        out["grad_rel_err"] = err
        if adj32 is not None:
            g32 = tuple(adj32.pop("grads")) + (None, None)
            adj32["grad_rel_err"] = summarise_along(along_errors(b, g32, idx, trajs, threads), 2000)[0]
            progress("FP32-backward gradient errors done")
    else:
        out["cpu_baseline"] = None
    if adj32 is not None:
        adj32.pop("grads", None)
    out["fp32_adjoint"] = adj32
    print(json.dumps(out))


if __name__ == "__main__":
    main()
