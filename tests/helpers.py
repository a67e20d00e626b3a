"""Shared test helpers: per-system errors, batched oracle calls, host
emulation bindings, GPU tensor helpers."""
from __future__ import annotations

import ctypes
import os

import numpy as np

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))

# Tolerances (per system, norm-wise: ||x - ref|| / max(||ref||, floor)).
TOL_QDD_F32 = 1e-5      # forward dynamics per step, FP32
TOL_STATE_F32 = 1e-3    # state after 1000 steps, FP32
TOL_GRAD_F32 = 1e-3     # gradients, FP32
FLOOR_F32 = 1e-6
FLOOR_F64 = 1e-12


def rel(x, ref, floor=FLOOR_F32):
    x, ref = np.asarray(x, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), floor))


def ball_tangent(s, q, gq):
    """The oracle's gradient gq along the unit sphere of every ball joint's
    quaternion (the form the library returns; oracle.ball_tangent)."""
    return O.ball_tangent(s, q, gq)


def split(vec, off):
    return [vec[..., off[i]:off[i + 1]] for i in range(len(off) - 1)]


def models(batch):
    return [O.Model(s, batch.gravity) for s in batch.systems]


def oracle_fd(batch, q, qd, tau):
    qo, vo, uo = batch.offsets()
    ms = models(batch)
    out = O.map_threads(lambda i: O.fd(ms[i], q[qo[i]:qo[i + 1]], qd[vo[i]:vo[i + 1]], tau[uo[i]:uo[i + 1]]),
                        range(len(ms)))
    return out


def oracle_grads(batch, gq_fn, gtraj=None, K=1, idx=None):
    """Per-system oracle (gq0, gqd0, gtau, qT, qdT); gq_fn(i, qT, qdT) gives
    the seeds (gqT, gqdT) of system i."""
    qo, vo, uo = batch.offsets()
    ms = models(batch)
    idx = range(len(ms)) if idx is None else idx

    def one(i):
        q0, qd0 = batch.q0[qo[i]:qo[i + 1]], batch.qd0[vo[i]:vo[i + 1]]
        tau = np.asarray(batch.tau[:, uo[i]:uo[i + 1]], dtype=np.float64)
        qT, qdT = O.rollout(ms[i], q0, qd0, tau, batch.dt)
        gqT, gqdT = gq_fn(i, qT, qdT)
        gt = None
        if gtraj is not None:
            gt = gtraj[i]
        return O.rollout_grad(ms[i], q0, qd0, tau, batch.dt, gqT, gqdT, gt, K=K)

    return O.map_threads(one, list(idx))


# ---------------------------------------------------------------- host emulation
_emu = None


def emu():
    global _emu
    if _emu is None:
        path = os.path.join(HERE, "hostemu", "libhostemu.so")
        csrc = os.path.join(HERE, "..", "paper_2109_07719_amd", "csrc")
        srcs = [os.path.join(HERE, "hostemu", "hostemu.cpp")] + [os.path.join(csrc, f) for f in
                                                                  ("aba_lane.h", "spatial.h")]
        if not os.path.exists(path) or os.path.getmtime(path) < max(os.path.getmtime(f) for f in srcs):
            import subprocess
            # parallel test workers may rebuild at once: each writes its own
            # file and renames it into place
            tmp = f"{path}.{os.getpid()}.tmp"
            subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wno-unknown-pragmas",
                                   "-o", tmp, os.path.join(HERE, "hostemu", "hostemu.cpp")])
            os.replace(tmp, path)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L.emu_fd_d.argtypes = [ctypes.c_int] + [P] * 8
        L.emu_fd_f.argtypes = [ctypes.c_int] + [P] * 8
        for n in ("emu_rollout_grad_d", "emu_rollout_grad_f"):
            getattr(L, n).argtypes = [ctypes.c_int] + [P] * 7 + [ctypes.c_double, ctypes.c_int] + [P] * 8
        _emu = L
    return _emu


def _axis_to_z(a):
    """Rotation R with R a = e_z (the library's joint-axis canonicalisation)."""
    a = np.asarray(a, dtype=np.float64)
    a = a / np.linalg.norm(a)
    c = a[2]
    if c > 1 - 1e-15:
        return np.eye(3)
    if c < -1 + 1e-15:
        return np.diag([1.0, -1.0, -1.0])
    k = np.array([a[1], -a[0], 0.0])
    sn = np.linalg.norm(k)
    k = k / sn
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + sn * K + (1 - c) * (K @ K)


def canonical_rotations(s):
    """Per link, the rotation Rl of the library's joint-axis canonicalisation
    (identity for a free root and a ball joint)."""
    return [np.eye(3) if s.jtype[i] in (1, 3) else _axis_to_z(s.axis[i]) for i in range(s.n)]


def frame_grad_to_user(s, acc):
    """Placement and axis gradients (phi_bar, r_T_bar, axis_bar) per link, in
    the caller's frames, from the accumulators in the kernels' canonical
    joint frames: xi (6) and w (3).  xi_user = [Rl^T xi_a; Rl^T xi_l];
    r_T_bar = E_T^T xi_user_l; the axis rotation adjoint is
    w_user = Rl^T (xi_a + w), and the axis gradient is w_user x a."""
    Rs = canonical_rotations(s)
    out = np.zeros((s.n, 9))
    for i in range(s.n):
        if s.jtype[i] == 1:
            continue
        R = Rs[i]
        if s.jtype[i] == 3:  # no axis: placement only
            out[i, 0:3] = acc[i, 0:3]
            out[i, 3:6] = np.asarray(s.E_T[i]).T @ acc[i, 3:6]
            continue
        xa, xl = R.T @ acc[i, 0:3], R.T @ acc[i, 3:6]
        a = np.asarray(s.axis[i], dtype=np.float64)
        a = a / np.linalg.norm(a)
        out[i, 0:3] = xa
        out[i, 3:6] = np.asarray(s.E_T[i]).T @ xl
        out[i, 6:9] = np.cross(R.T @ (acc[i, 0:3] + acc[i, 6:9]), a)
    return out


def link_constants(s):
    """The 25 per-link constants in the kernels' order after the library's
    joint-axis canonicalisation (every link frame rotated so that its joint
    axis is e_z): E_T' = Rl E_T Rp^T, r_T' = Rp r_T, axis' = e_z, m, m*c',
    inertia about the link origin (xx yy zz xy xz yz) with c' = Rl c,
    Ic' = Rl Ic Rl^T."""
    n = s.n
    Rs = canonical_rotations(s)
    cf = np.zeros((n, 25))
    for i in range(n):
        Rl = Rs[i]
        Rp = np.eye(3) if s.parent[i] < 0 else Rs[s.parent[i]]
        cf[i, 0:9] = (Rl @ np.asarray(s.E_T[i]) @ Rp.T).reshape(9)
        cf[i, 9:12] = Rp @ np.asarray(s.r_T[i])
        cf[i, 12:15] = [0.0, 0.0, 1.0]
        m = float(s.mass[i])
        c = Rl @ np.asarray(s.com[i], dtype=np.float64)
        Ic = np.asarray(s.Ic[i], dtype=np.float64)
        J = np.array([[Ic[0], Ic[3], Ic[4]], [Ic[3], Ic[1], Ic[5]], [Ic[4], Ic[5], Ic[2]]])
        J = Rl @ J @ Rl.T
        cf[i, 15] = m
        cf[i, 16:19] = m * c
        cf[i, 19] = J[0, 0] + m * (c[1] ** 2 + c[2] ** 2)
        cf[i, 20] = J[1, 1] + m * (c[0] ** 2 + c[2] ** 2)
        cf[i, 21] = J[2, 2] + m * (c[0] ** 2 + c[1] ** 2)
        cf[i, 22] = J[0, 1] - m * c[0] * c[1]
        cf[i, 23] = J[0, 2] - m * c[0] * c[2]
        cf[i, 24] = J[1, 2] - m * c[1] * c[2]
    return np.ascontiguousarray(cf)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def emu_fd(s, q, qd, tau, gravity=(0.0, -9.81, 0.0), f32=False):
    dt = np.float32 if f32 else np.float64
    par = np.ascontiguousarray(s.parent, np.int32)
    jt = np.ascontiguousarray(s.jtype, np.int32)
    cf, g = link_constants(s), np.ascontiguousarray(gravity, np.float64)
    q, qd, tau = (np.ascontiguousarray(x, dt) for x in (q, qd, tau))
    out = np.zeros(s.nv, dt)
    (emu().emu_fd_f if f32 else emu().emu_fd_d)(s.n, _p(par), _p(jt), _p(cf), _p(g), _p(q), _p(qd), _p(tau),
                                                _p(out))
    return out


def emu_rollout_grad(s, q0, qd0, tau, dt_, gqT, gqdT, gravity=(0.0, -9.81, 0.0), f32=False, frame=False):
    dt = np.float32 if f32 else np.float64
    par = np.ascontiguousarray(s.parent, np.int32)
    jt = np.ascontiguousarray(s.jtype, np.int32)
    cf, g = link_constants(s), np.ascontiguousarray(gravity, np.float64)
    T = int(np.asarray(tau).shape[0])
    q0, qd0, tau, gqT, gqdT = (np.ascontiguousarray(x, dt) for x in (q0, qd0, tau, gqT, gqdT))
    gq0, gqd0 = np.zeros(s.nq, dt), np.zeros(s.nv, dt)
    gtau = np.zeros((T, s.nu), dt)
    qT, qdT = np.zeros(s.nq, dt), np.zeros(s.nv, dt)
    acc = np.zeros((s.n, 9), dt)
    (emu().emu_rollout_grad_f if f32 else emu().emu_rollout_grad_d)(
        s.n, _p(par), _p(jt), _p(cf), _p(g), _p(q0), _p(qd0), _p(tau), float(dt_), T, _p(gqT), _p(gqdT),
        _p(gq0), _p(gqd0), _p(gtau), _p(qT), _p(qdT), _p(acc) if frame else None)
    if frame:
        return gq0, gqd0, gtau, qT, qdT, frame_grad_to_user(s, acc.astype(np.float64))
    return gq0, gqd0, gtau, qT, qdT


_cemu = None


def contact_emu():
    """Host build of the GPU contact step (tests/hostemu/contact_emu.cpp)."""
    global _cemu
    if _cemu is None:
        path = os.path.join(HERE, "hostemu", "libcontactemu.so")
        src = os.path.join(HERE, "hostemu", "contact_emu.cpp")
        csrc = os.path.join(HERE, "..", "paper_2109_07719_amd", "csrc")
        deps = [src] + [os.path.join(csrc, f) for f in ("contact_step.h", "contact_adjoint.h", "dual.h", "spatial.h")]
        if not os.path.exists(path) or os.path.getmtime(path) < max(os.path.getmtime(f) for f in deps):
            import subprocess
            tmp = f"{path}.{os.getpid()}.tmp"
            subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wno-unknown-pragmas",
                                   "-o", tmp, src])
            os.replace(tmp, path)
        L = ctypes.CDLL(path)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.emu_contact_rollout.argtypes = [I, I, P, P, I, P, D, D, I, P, P, P, P, P, D, I, P, P, P, I]
        L.emu_contact_grad.argtypes = [I, I, P, P, I, P, D, D, I, P, P, P, P, D, I, P, P, P, P, P, P, P]
        L.emu_contact_grad_adj.argtypes = [I, I, P, P, I, P, D, D, I, P, P, P, P, D, I, P, P, P, P, P, P, P, I]
        _cemu = L
    return _cemu
