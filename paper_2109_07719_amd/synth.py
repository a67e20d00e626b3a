"""Seeded synthetic articulated systems and inputs.

This module only draws random numbers and lays out geometry; it contains none
of the dynamics.  Both the GPU path and the CPU oracle consume the arrays it
produces, so that parity runs compare the two on identical inputs.

The paper's scenes (the Laikago quadruped of Sec. 6.1, the MuJoCo Ant of
Sec. 6.2) are not available; the workloads below stand in for them with the
same dimensional profile (Sec. 6.1: 19 position and 18 velocity dimensions
for the quadruped).

Conventions shared with the rest of the package:
  * per link: parent index local to the system (-1 = fixed base / none),
    joint type (0 revolute, 1 free, 2 prismatic, 3 spherical; free only at local index 0), fixed
    rotation E_T (3x3, parent -> joint frame), joint origin r_T in parent
    coordinates, unit joint axis, mass, centre of mass, rotational inertia
    about the COM as (xx, yy, zz, xy, xz, yz);
  * q of a free root is (p_world[3], quat[4] as x, y, z, w), its velocity the
    body-frame spatial velocity [w; v]; the root is unactuated;
  * batched vectors are system-concatenated; tau is [T][sum nu].

Every generator draws from ``numpy.random.default_rng(seed)`` in float64;
GPU runs use the float32-rounded values and the oracle the same rounded
values widened back to float64.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

REVOLUTE = 0
FREE = 1
PRISMATIC = 2
SPHERICAL = 3
GRAVITY = np.array([0.0, -9.81, 0.0])


@dataclass
class System:
    """One articulated tree (links in topological order: parent < child)."""

    parent: np.ndarray
    jtype: np.ndarray
    E_T: np.ndarray
    r_T: np.ndarray
    axis: np.ndarray
    mass: np.ndarray
    com: np.ndarray
    Ic: np.ndarray
    # optional joint limits [n, 4]: lo, hi, stiffness k, damping d of the
    # one-sided spring-damper that acts outside [lo, hi] (1-dof joints)
    limits: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.parent.shape[0])

    @property
    def nq(self) -> int:
        return int(np.sum(np.select([self.jtype == FREE, self.jtype == SPHERICAL], [7, 4], 1)))

    @property
    def nv(self) -> int:
        return int(np.sum(np.select([self.jtype == FREE, self.jtype == SPHERICAL], [6, 3], 1)))

    @property
    def nu(self) -> int:
        return int(np.sum(np.select([self.jtype == FREE, self.jtype == SPHERICAL], [0, 3], 1)))

    def depth(self) -> np.ndarray:
        d = np.zeros(self.n, dtype=np.int64)
        for i in range(self.n):
            d[i] = 0 if self.parent[i] < 0 else d[self.parent[i]] + 1
        return d


@dataclass
class Batch:
    """A batch of systems with initial states and a control sequence."""

    systems: list
    q0: np.ndarray          # [sum nq] float64
    qd0: np.ndarray         # [sum nv] float64
    tau: np.ndarray         # [T][sum nu] (float32 or float64)
    dt: float
    gravity: np.ndarray = field(default_factory=lambda: GRAVITY.copy())
    name: str = ""

    @property
    def T(self) -> int:
        return int(self.tau.shape[0])

    def offsets(self):
        """Per-system offsets into q, qd and tau vectors."""
        nq = np.array([s.nq for s in self.systems])
        nv = np.array([s.nv for s in self.systems])
        nu = np.array([s.nu for s in self.systems])
        z = np.zeros(1, dtype=np.int64)
        return (np.concatenate([z, np.cumsum(nq)]), np.concatenate([z, np.cumsum(nv)]),
                np.concatenate([z, np.cumsum(nu)]))

    @property
    def total_dof(self) -> int:
        return int(sum(s.nv for s in self.systems))


def _eye(n):
    return np.broadcast_to(np.eye(3), (n, 3, 3)).copy()


def _unit(v):
    return v / np.linalg.norm(v)


# --------------------------------------------------------------------------
# serial chains (7-DOF chain workloads, trajectory-optimisation chains)
# --------------------------------------------------------------------------

def chain_geometry(n: int, mass: np.ndarray, Icd: np.ndarray) -> System:
    """Fixed-base serial chain of revolute joints about z, links 0.5 m apart,
    COM at (0.25, 0, 0) in each link frame, diagonal inertias."""
    r_T = np.zeros((n, 3))
    r_T[1:, 0] = 0.5
    axis = np.zeros((n, 3))
    axis[:, 2] = 1.0
    com = np.zeros((n, 3))
    com[:, 0] = 0.25
    Ic = np.zeros((n, 6))
    Ic[:, :3] = Icd
    return System(parent=np.arange(-1, n - 1, dtype=np.int32),
                  jtype=np.zeros(n, dtype=np.int32), E_T=_eye(n), r_T=r_T,
                  axis=axis, mass=mass, com=com, Ic=Ic)


def chain_system(n: int, seed: int, T: int):
    """Draw order: masses U(0.5, 2); inertia diagonals U(0.01, 0.1) (3 per
    link); q0, qd0 ~ N(0, 0.1^2); tau ~ N(0, 1) [T x n]."""
    rng = np.random.default_rng(seed)
    mass = rng.uniform(0.5, 2.0, n)
    Icd = rng.uniform(0.01, 0.1, (n, 3))
    q0 = rng.normal(0.0, 0.1, n)
    qd0 = rng.normal(0.0, 0.1, n)
    tau = rng.normal(0.0, 1.0, (T, n))
    return chain_geometry(n, mass, Icd), q0, qd0, tau


# --------------------------------------------------------------------------
# uneven branched trees
# --------------------------------------------------------------------------

def tree_system(seed: int, T: int, nmin: int = 6, nmax: int = 40,
                max_depth: int = 6, random_frames: bool = False, prismatic: float = 0.0):
    """Fixed-base tree: n ~ U{nmin..nmax}; breadth-first growth where every
    node below the depth limit gets b ~ U{1,2,3} children; the first n nodes
    in BFS order are kept (the growth is redrawn if fewer than n exist).
    Axes normalize(N(0, I3)); r_T = 0.5 * random unit vector; COM ~
    U[-0.25, 0.25]^3; masses and inertias as for chains; q0, qd0 ~
    N(0, 0.1^2); tau ~ N(0, 1).  With random_frames, E_T is a random
    rotation (not part of the benchmark workload; used to widen tests).
    With prismatic > 0, every joint becomes prismatic with that probability,
    drawn from a separate stream (seed + 10^6) so that the other draws are
    unchanged."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(nmin, nmax + 1))
    while True:
        parent = [-1]
        depth = [1]
        head = 0
        while head < len(parent) and len(parent) < n:
            if depth[head] < max_depth:
                b = int(rng.integers(1, 4))
                for _ in range(b):
                    if len(parent) < n:
                        parent.append(head)
                        depth.append(depth[head] + 1)
            head += 1
        if len(parent) == n:
            break
    parent = np.array(parent, dtype=np.int32)
    axis = np.stack([_unit(rng.normal(size=3)) for _ in range(n)])
    r_T = np.stack([0.5 * _unit(rng.normal(size=3)) for _ in range(n)])
    com = rng.uniform(-0.25, 0.25, (n, 3))
    mass = rng.uniform(0.5, 2.0, n)
    Icd = rng.uniform(0.01, 0.1, (n, 3))
    Ic = np.zeros((n, 6))
    Ic[:, :3] = Icd
    E_T = _eye(n)
    if random_frames:
        for i in range(n):
            qq = _unit(rng.normal(size=4))
            x, y, z, w = qq
            E_T[i] = np.array([
                [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
    q0 = rng.normal(0.0, 0.1, n)
    qd0 = rng.normal(0.0, 0.1, n)
    tau = rng.normal(0.0, 1.0, (T, n))
    jtype = np.zeros(n, dtype=np.int32)
    if prismatic > 0:
        jtype[np.random.default_rng(seed + 1_000_000).uniform(size=n) < prismatic] = PRISMATIC
    sys_ = System(parent=parent, jtype=jtype, E_T=E_T,
                  r_T=r_T, axis=axis, mass=mass, com=com, Ic=Ic)
    return sys_, q0, qd0, tau


def cartpole_system(seed: int, T: int):
    """A cart sliding along x (prismatic root, axis (1, 0, 0)) carrying a
    pole on a z-axis revolute joint at the cart origin; pole COM (l, 0, 0)
    with l ~ U(0.3, 0.8); cart mass U(0.5, 2), pole mass U(0.1, 0.5), pole
    inertias U(0.001, 0.01); q0, qd0 ~ N(0, 0.1^2); tau ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    l = rng.uniform(0.3, 0.8)
    mass = np.array([rng.uniform(0.5, 2.0), rng.uniform(0.1, 0.5)])
    Ic = np.zeros((2, 6))
    Ic[:, :3] = rng.uniform(0.001, 0.01, (2, 3))
    com = np.array([[0.0, 0.0, 0.0], [l, 0.0, 0.0]])
    axis = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    sys_ = System(parent=np.array([-1, 0], dtype=np.int32), jtype=np.array([PRISMATIC, REVOLUTE], dtype=np.int32),
                  E_T=_eye(2), r_T=np.zeros((2, 3)), axis=axis, mass=mass, com=com, Ic=Ic)
    return sys_, rng.normal(0.0, 0.1, 2), rng.normal(0.0, 0.1, 2), rng.normal(0.0, 1.0, (T, 2))


# --------------------------------------------------------------------------
# quadruped: free-floating base + 4 legs x 3 revolute joints
# --------------------------------------------------------------------------

def quadruped_system(seed: int, T: int):
    """10 kg box base (0.6 x 0.15 x 0.3 m) on a free joint; legs at hips
    (+-0.25, 0, +-0.1) with joint axes x, z, z; thigh and calf 0.25 m long
    along -y with COM at mid-link.  Draw order: leg masses U(0.3, 1.5) (12);
    leg inertia diagonals U(0.001, 0.01) (12 x 3); joint q ~ N(0, 0.1^2)
    (12); velocities ~ N(0, 0.1^2) (18); tau ~ N(0, 1) [T x 12].  Base at
    p = (0, 0.5, 0) with identity orientation.  No contact: free fall."""
    rng = np.random.default_rng(seed)
    leg_mass = rng.uniform(0.3, 1.5, 12)
    leg_Icd = rng.uniform(0.001, 0.01, (12, 3))
    n = 13
    parent = np.full(n, -1, dtype=np.int32)
    jtype = np.zeros(n, dtype=np.int32)
    jtype[0] = FREE
    r_T = np.zeros((n, 3))
    axis = np.zeros((n, 3))
    com = np.zeros((n, 3))
    mass = np.zeros(n)
    Ic = np.zeros((n, 6))
    a, b, c = 0.6, 0.15, 0.3
    mass[0] = 10.0
    Ic[0, :3] = [10.0 / 12 * (b * b + c * c), 10.0 / 12 * (a * a + c * c), 10.0 / 12 * (a * a + b * b)]
    axis[0] = [0.0, 0.0, 1.0]  # unused for the free joint
    k = 1
    for leg, (sx, sz) in enumerate([(1, 1), (1, -1), (-1, 1), (-1, -1)]):
        hip, thigh, calf = k, k + 1, k + 2
        parent[hip], parent[thigh], parent[calf] = 0, hip, thigh
        r_T[hip] = [0.25 * sx, 0.0, 0.1 * sz]
        r_T[thigh] = [0.0, 0.0, 0.0]
        r_T[calf] = [0.0, -0.25, 0.0]
        axis[hip] = [1.0, 0.0, 0.0]
        axis[thigh] = [0.0, 0.0, 1.0]
        axis[calf] = [0.0, 0.0, 1.0]
        com[hip] = [0.0, 0.0, 0.0]
        com[thigh] = [0.0, -0.125, 0.0]
        com[calf] = [0.0, -0.125, 0.0]
        for j, li in enumerate((hip, thigh, calf)):
            mass[li] = leg_mass[3 * leg + j]
            Ic[li, :3] = leg_Icd[3 * leg + j]
        k += 3
    qj = rng.normal(0.0, 0.1, 12)
    v = rng.normal(0.0, 0.1, 18)
    tau = rng.normal(0.0, 1.0, (T, 12))
    q0 = np.concatenate([[0.0, 0.5, 0.0, 0.0, 0.0, 0.0, 1.0], qj])
    sys_ = System(parent=parent, jtype=jtype, E_T=_eye(n), r_T=r_T, axis=axis,
                  mass=mass, com=com, Ic=Ic)
    return sys_, q0, v, tau



def landing_quadruped(seed: int, T: int, drop: float = 0.005):
    """Contact workload: quadruped_system(seed, T) with a contact sphere of
    radius 0.03 at each calf's end (0, -0.25, 0), the base lowered so that
    the feet start `drop` above the ground plane y = 0, torques scaled by
    0.3.  It falls, lands on its feet, and the legs then fold under the
    random torques with 2-4 feet on the ground (only the feet carry
    spheres).  Returns (system, q0, qd0, tau, contact links, centres,
    radii)."""
    s, q0, qd0, tau = quadruped_system(seed, T)
    q0 = q0.copy()
    q0[1] = 0.5 + 0.03 + drop
    links = np.array([3, 6, 9, 12], np.int32)
    centers = np.tile([0.0, -0.25, 0.0], (4, 1))
    radii = np.full(4, 0.03)
    return s, q0, qd0, 0.3 * tau, links, centers, radii

def telescoping_quadruped_system(seed: int, T: int):
    """quadruped_system(seed, T) with every knee replaced by a prismatic
    joint sliding along the leg (axis (0, 1, 0)): a free-floating base over
    revolute and prismatic joints.  Same draws as quadruped_system."""
    sys_, q0, v, tau = quadruped_system(seed, T)
    jtype = sys_.jtype.copy()
    axis = sys_.axis.copy()
    for calf in (3, 6, 9, 12):
        jtype[calf] = PRISMATIC
        axis[calf] = [0.0, 1.0, 0.0]
    return replace(sys_, jtype=jtype, axis=axis), q0, v, tau


def with_spherical_joints(sys_: System, q0, qd0, tau, links, seed: int):
    """The system with the joints of the given links turned into spherical
    (ball) joints, and its state and controls re-laid out: such a joint's q
    entry becomes a unit quaternion (x, y, z, w) of a rotation vector ~
    N(0, 0.3^2), its qd entry a link-frame angular velocity ~ N(0, 0.3^2)
    (3), its tau entry three torques ~ N(0, 1).  The new draws come from
    their own stream (seed); every other entry keeps its value."""
    rng = np.random.default_rng(seed)
    links = set(int(i) for i in links)
    jtype = sys_.jtype.copy()
    T = tau.shape[0]
    q, qd, u = [], [], []
    qi = vi = ui = 0
    for i in range(sys_.n):
        if jtype[i] == FREE:
            q.append(q0[qi:qi + 7]); qd.append(qd0[vi:vi + 6])
            qi += 7; vi += 6
            continue
        if i in links:
            w = rng.normal(0.0, 0.3, 3)
            th = float(np.linalg.norm(w))
            quat = np.r_[np.sin(th / 2) * w / th, np.cos(th / 2)] if th > 0 else np.array([0.0, 0.0, 0.0, 1.0])
            q.append(quat); qd.append(rng.normal(0.0, 0.3, 3)); u.append(rng.normal(0.0, 1.0, (T, 3)))
            jtype[i] = SPHERICAL
        else:
            q.append(q0[qi:qi + 1]); qd.append(qd0[vi:vi + 1]); u.append(tau[:, ui:ui + 1])
        qi += 1; vi += 1; ui += 1
    tau_new = np.concatenate(u, axis=1) if u else np.zeros((T, 0))
    return replace(sys_, jtype=jtype), np.concatenate(q), np.concatenate(qd), tau_new


def ball_tree_system(seed: int, T: int, spherical: float = 0.3, **kw):
    """tree_system(seed, T, **kw) with every joint spherical with the given
    probability (drawn from the stream seed + 2 * 10^6, which also draws the
    new joints' states and torques)."""
    sys_, q0, qd0, tau = tree_system(seed, T, **kw)
    pick = np.random.default_rng(seed + 2_000_000).uniform(size=sys_.n) < spherical
    return with_spherical_joints(sys_, q0, qd0, tau, np.nonzero(pick)[0], seed + 3_000_000)


def ball_quadruped_system(seed: int, T: int):
    """quadruped_system(seed, T) with every hip a ball joint: a free-floating
    base over spherical hips and revolute thighs and knees (n_q = 31, n_v =
    26, 20 controls).  Same draws as quadruped_system, then the ball joints'
    from the stream seed + 3 * 10^6."""
    sys_, q0, v, tau = quadruped_system(seed, T)
    return with_spherical_joints(sys_, q0, v, tau, (1, 4, 7, 10), seed + 3_000_000)


def prismatic_chain_system(n: int, seed: int, T: int):
    """chain_system(n, seed, T) with every third joint (local index 2, 5,
    ...) prismatic, sliding along the link (axis (1, 0, 0)): a serial chain
    that is not all revolute.  Same draws as chain_system."""
    sys_, q0, qd0, tau = chain_system(n, seed, T)
    jtype = sys_.jtype.copy()
    axis = sys_.axis.copy()
    jtype[2::3] = PRISMATIC
    axis[2::3] = [1.0, 0.0, 0.0]
    return replace(sys_, jtype=jtype, axis=axis), q0, qd0, tau


def with_joint_limits(draw, seed: int, half_range=(0.05, 0.3), k=(100.0, 400.0), d=(0.5, 3.0)):
    """The same (system, q0, qd0, tau) with limits on every 1-dof joint: a
    range [q0_i - w_i, q0_i + w_i] around its start, w ~ U(half_range),
    stiffness k ~ U(k), damping d ~ U(d) (drawn from seed), so that
    rollouts under gravity and the random torques run into them."""
    s, q0, qd0, tau = draw
    rng = np.random.default_rng(seed)
    lim = np.zeros((s.n, 4))
    qi = 0
    for i in range(s.n):
        if s.jtype[i] == FREE:
            lim[i] = [-1e30, 1e30, 0.0, 0.0]
            qi += 7
            continue
        w = rng.uniform(*half_range)
        lim[i] = [q0[qi] - w, q0[qi] + w, rng.uniform(*k), rng.uniform(*d)]
        qi += 1
    return replace(s, limits=lim), q0, qd0, tau


# --------------------------------------------------------------------------
# batches
# --------------------------------------------------------------------------

def make_batch(draws, dt: float, name: str = "", tau_dtype=np.float64) -> Batch:
    systems = [d[0] for d in draws]
    T = draws[0][3].shape[0]
    nu_tot = sum(s.nu for s in systems)
    tau = np.empty((T, nu_tot), dtype=tau_dtype)
    off = 0
    for s, _, _, t in draws:
        tau[:, off:off + s.nu] = t
        off += s.nu
    q0 = np.concatenate([d[1] for d in draws]).astype(np.float64)
    qd0 = np.concatenate([d[2] for d in draws]).astype(np.float64)
    return Batch(systems=systems, q0=q0, qd0=qd0, tau=tau, dt=dt, name=name)


def round_to_f32(b: Batch) -> Batch:
    """Round every floating input to float32 and widen back (the oracle's view
    of what the float32 GPU path consumes), the step size and gravity
    included."""
    def r(x):
        return np.asarray(x, dtype=np.float32).astype(np.float64)
    systems = [System(parent=s.parent, jtype=s.jtype, E_T=r(s.E_T), r_T=r(s.r_T),
                      axis=r(s.axis), mass=r(s.mass), com=r(s.com), Ic=r(s.Ic),
                      limits=None if s.limits is None else r(s.limits))
               for s in b.systems]
    return Batch(systems=systems, q0=r(b.q0), qd0=r(b.qd0), tau=r(b.tau), dt=float(np.float32(b.dt)),
                 gravity=r(b.gravity), name=b.name)


def workload(name: str, n_systems: int | None = None, T: int | None = None,
             tau_dtype=np.float64) -> Batch:
    """The workloads by name:
      chain7_fp64   1 chain of 7 revolute joints, seed 0, dt 1e-3, T 1000
      chain7_4096   4096 such chains (seed 1000+i), dt 1e-3, T 5000
      trees_8192    8192 uneven trees of 6-40 links, depth <= 6 (seed 2000+i),
                    dt 5e-4, T 2000
      quad_1024     1024 quadrupeds (seed 3000+i), dt 1e-3, T 50000
      chains_2048   2048 chains of 5-50 links (seed 4000+i), dt 1e-3, T 1000,
                    q0 = qd0 = 0 and tau = 0 (optimisation start)
      trees_prismatic_8192
                    the trees_8192 systems with each joint prismatic with
                    probability 0.3 (same shapes and draws otherwise)
      ball_quad_1024
                    1024 quadrupeds on ball hips (ball_quadruped_system,
                    seed 3000+i), dt 1e-3, T 2000 (under these random
                    torques the ball hips spin up and the rollouts diverge
                    after 5000-20000 steps, in the oracle alike)
    n_systems / T shrink a workload for tests (the seeds stay the same)."""
    if name == "chain7_fp64":
        ns, TT, dt = 1, 1000, 1e-3
        ns, TT = n_systems or ns, T or TT
        draws = [chain_system(7, 0 + i, TT) for i in range(ns)]
    elif name == "chain7_4096":
        ns, TT, dt = 4096, 5000, 1e-3
        ns, TT = n_systems or ns, T or TT
        draws = [chain_system(7, 1000 + i, TT) for i in range(ns)]
    elif name == "trees_8192":
        ns, TT, dt = 8192, 2000, 5e-4
        ns, TT = n_systems or ns, T or TT
        draws = [tree_system(2000 + i, TT) for i in range(ns)]
    elif name == "trees_prismatic_8192":
        ns, TT, dt = 8192, 2000, 5e-4
        ns, TT = n_systems or ns, T or TT
        draws = [tree_system(2000 + i, TT, prismatic=0.3) for i in range(ns)]
    elif name == "quad_1024":
        ns, TT, dt = 1024, 50000, 1e-3
        ns, TT = n_systems or ns, T or TT
        draws = [quadruped_system(3000 + i, TT) for i in range(ns)]
    elif name == "ball_quad_1024":
        ns, TT, dt = 1024, 2000, 1e-3
        ns, TT = n_systems or ns, T or TT
        draws = [ball_quadruped_system(3000 + i, TT) for i in range(ns)]
    elif name == "chains_2048":
        ns, TT, dt = 2048, 1000, 1e-3
        ns, TT = n_systems or ns, T or TT
        draws = []
        for i in range(ns):
            rng = np.random.default_rng(4000 + i)
            n = int(rng.integers(5, 51))
            mass = rng.uniform(0.5, 2.0, n)
            Icd = rng.uniform(0.01, 0.1, (n, 3))
            draws.append((chain_geometry(n, mass, Icd), np.zeros(n), np.zeros(n),
                          np.zeros((TT, n))))
    else:
        raise ValueError(f"unknown workload {name!r}")
    return make_batch(draws, dt, name=name, tau_dtype=tau_dtype)


def chains_targets(n_systems: int, seed0: int = 4000):
    """Random joint configurations q* ~ U(-pi, pi)^n for the optimisation
    chains (drawn after the chain parameters, from the same seeds); the
    end-effector targets are the end-effector positions of q*."""
    out = []
    for i in range(n_systems):
        rng = np.random.default_rng(seed0 + i)
        n = int(rng.integers(5, 51))
        rng.uniform(0.5, 2.0, n)
        rng.uniform(0.01, 0.1, (n, 3))
        out.append(rng.uniform(-np.pi, np.pi, n))
    return out
