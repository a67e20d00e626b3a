"""Independent textbook dynamics used to pin the oracle (test helper).

Classical recursive Newton-Euler in WORLD coordinates with plain 3-vectors
and rotation matrices -- deliberately a different formalism from the spatial
(6-D Plucker) algebra used by both the oracle and the GPU path, so that a
convention or sign slip there cannot be mirrored here.  Works for real and
complex arrays (complex-step derivatives of inverse dynamics).

  ID(q, qd, qdd) = tau   (joint torques; for a free root the first six
                          entries are the net body-frame wrench [n; f] that
                          must vanish for free motion)
  M(q) columns   = ID(q, 0, e_j) - ID(q, 0, 0)
  FD(q, qd, tau) = M^{-1} (tau - ID(q, qd, 0))

Joint kinematics follow the package convention: a link frame is reached from
its parent by the fixed rotation E_T and offset r_T, then a rotation by q
about the unit axis a (coordinates map by E = E_J(q) E_T, so the
link-to-parent rotation matrix is E^T), or, for a prismatic joint (type 2),
a translation by q along a, or, for a spherical joint (type 3), the rotation
of the unit quaternion q (x, y, z, w) with the link's angular velocity
relative to its parent given in link coordinates (3 velocity entries and 3
torque entries, the torque about the link origin in link coordinates).
"""
from __future__ import annotations

import numpy as np


def _rot_axis(a, q):
    """Rotation matrix (link -> pre-joint frame) of angle q about unit a."""
    a = np.asarray(a, dtype=float)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(q) * K + (1 - np.cos(q)) * (K @ K)


def _quat_R(qt):
    x, y, z, w = qt
    return np.array([
        [w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z]])


def _Icom(Ic):
    xx, yy, zz, xy, xz, yz = Ic
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def kinematics(sys_, q, qd, qdd, gravity):
    """World-frame positions, rotations, angular velocities/accelerations and
    linear accelerations of each link origin.  Returns per-link lists."""
    n = sys_.n
    dt = np.result_type(q, qd, qdd, float)
    R = [None] * n
    o = [None] * n
    w = [None] * n
    wd = [None] * n
    vo = [None] * n
    ao = [None] * n
    z = [None] * n
    k = 0
    kv = 0
    for i in range(n):
        lam = sys_.parent[i]
        if sys_.jtype[i] == 1:
            p = q[k:k + 3]
            qt = q[k + 3:k + 7]
            Ri = _quat_R(qt)
            wb, vb = qd[kv:kv + 3], qd[kv + 3:kv + 6]
            wbd, vbd = qdd[kv:kv + 3], qdd[kv + 3:kv + 6]
            R[i], o[i] = Ri, p
            w[i] = Ri @ wb
            wd[i] = Ri @ wbd
            vo[i] = Ri @ vb
            ao[i] = Ri @ vbd + np.cross(w[i], vo[i])
            z[i] = None
            k += 7
            kv += 6
            continue
        if lam < 0:
            Rl, ol = np.eye(3, dtype=dt), np.zeros(3, dtype=dt)
            wl, wdl = np.zeros(3, dtype=dt), np.zeros(3, dtype=dt)
            vl, al = np.zeros(3, dtype=dt), np.zeros(3, dtype=dt)
        else:
            Rl, ol, wl, wdl, vl, al = R[lam], o[lam], w[lam], wd[lam], vo[lam], ao[lam]
        ET = np.asarray(sys_.E_T[i], dtype=float)
        a = np.asarray(sys_.axis[i], dtype=float)
        Rpre = Rl @ ET.T                # pre-joint frame -> world
        zi = Rpre @ a                   # world joint axis
        if sys_.jtype[i] == 3:
            # spherical: a ball joint at the joint origin
            rij = Rl @ np.asarray(sys_.r_T[i], dtype=float)
            oi = ol + rij
            Ri = Rpre @ _quat_R(q[k:k + 4])
            wrel = Ri @ qd[kv:kv + 3]
            wi = wl + wrel
            wdi = wdl + Ri @ qdd[kv:kv + 3] + np.cross(wl, wrel)
            voi = vl + np.cross(wl, rij)
            aoi = al + np.cross(wdl, rij) + np.cross(wl, np.cross(wl, rij))
            R[i], o[i], w[i], wd[i], vo[i], ao[i], z[i] = Ri, oi, wi, wdi, voi, aoi, None
            k += 4
            kv += 3
            continue
        if sys_.jtype[i] == 2:
            # prismatic: the link origin slides by q along the axis, no rotation
            rij = Rl @ np.asarray(sys_.r_T[i], dtype=float) + zi * q[k]
            oi = ol + rij
            Ri = Rpre
            wi, wdi = wl, wdl
            voi = vl + np.cross(wl, rij) + zi * qd[kv]
            aoi = (al + np.cross(wdl, rij) + np.cross(wl, np.cross(wl, rij)) + 2 * np.cross(wl, zi) * qd[kv]
                   + zi * qdd[kv])
        else:
            rij = Rl @ np.asarray(sys_.r_T[i], dtype=float)
            oi = ol + rij
            Ri = Rpre @ _rot_axis(a, q[k])  # link frame -> world
            wi = wl + zi * qd[kv]
            wdi = wdl + zi * qdd[kv] + np.cross(wl, zi) * qd[kv]
            voi = vl + np.cross(wl, rij)
            aoi = al + np.cross(wdl, rij) + np.cross(wl, np.cross(wl, rij))
        R[i], o[i], w[i], wd[i], vo[i], ao[i], z[i] = Ri, oi, wi, wdi, voi, aoi, zi
        k += 1
        kv += 1
    return R, o, w, wd, vo, ao, z


def inverse_dynamics(sys_, q, qd, qdd, gravity=(0.0, -9.81, 0.0)):
    g = np.asarray(gravity, dtype=float)
    n = sys_.n
    R, o, w, wd, vo, ao, z = kinematics(sys_, q, qd, qdd, g)
    F = [None] * n
    N = [None] * n
    pc = [None] * n
    for i in range(n):
        c = R[i] @ np.asarray(sys_.com[i], dtype=float)
        pc[i] = o[i] + c
        ac = ao[i] + np.cross(wd[i], c) + np.cross(w[i], np.cross(w[i], c))
        m = float(sys_.mass[i])
        Iw = R[i] @ _Icom(sys_.Ic[i]) @ R[i].T
        F[i] = m * (ac - g)
        N[i] = Iw @ wd[i] + np.cross(w[i], Iw @ w[i])
    f = [F[i].copy() for i in range(n)]
    nm = [N[i] + np.cross(pc[i] - o[i], F[i]) for i in range(n)]
    for i in range(n - 1, -1, -1):
        lam = sys_.parent[i]
        if lam >= 0:
            f[lam] = f[lam] + f[i]
            nm[lam] = nm[lam] + nm[i] + np.cross(o[i] - o[lam], f[i])
    out = []
    for i in range(n):
        if sys_.jtype[i] == 1:
            out.extend(list(R[i].T @ nm[i]) + list(R[i].T @ f[i]))
        elif sys_.jtype[i] == 3:
            out.extend(list(R[i].T @ nm[i]))
        elif sys_.jtype[i] == 2:
            out.append(z[i] @ f[i])
        else:
            out.append(z[i] @ nm[i])
    return np.array(out)


def mass_matrix(sys_, q, gravity=(0.0, -9.81, 0.0)):
    nv = sys_.nv
    z = np.zeros(nv)
    bias = inverse_dynamics(sys_, q, z, z, gravity)
    M = np.zeros((nv, nv))
    for j in range(nv):
        e = np.zeros(nv)
        e[j] = 1.0
        M[:, j] = inverse_dynamics(sys_, q, z, e, gravity) - bias
    return M


def forward_dynamics(sys_, q, qd, tau, gravity=(0.0, -9.81, 0.0)):
    nv = sys_.nv
    M = mass_matrix(sys_, q, gravity)
    C = inverse_dynamics(sys_, q, qd, np.zeros(nv), gravity)
    tau = np.asarray(tau, dtype=float)
    full_tau = np.concatenate([np.zeros(6), tau]) if sys_.jtype[0] == 1 else tau
    return np.linalg.solve(M, full_tau - C)


def energy(sys_, q, qd, gravity=(0.0, -9.81, 0.0)):
    """Kinetic + potential energy from world-frame link velocities."""
    g = np.asarray(gravity, dtype=float)
    R, o, w, wd, vo, ao, z = kinematics(sys_, q, qd, np.zeros_like(qd), g)
    E = 0.0
    for i in range(sys_.n):
        c = R[i] @ np.asarray(sys_.com[i], dtype=float)
        vc = vo[i] + np.cross(w[i], c)
        m = float(sys_.mass[i])
        Iw = R[i] @ _Icom(sys_.Ic[i]) @ R[i].T
        E += 0.5 * m * vc @ vc + 0.5 * w[i] @ Iw @ w[i] - m * g @ (o[i] + c)
    return E
