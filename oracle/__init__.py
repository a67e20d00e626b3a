"""Python access to the plain FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use it; the product path never does.  This wrapper
imports nothing from the GPU package: systems are passed as any object with
the attributes parent, jtype, E_T, r_T, axis, mass, com, Ic (numpy arrays).

ctypes releases the GIL during foreign calls, so ``map_threads`` runs
independent systems on several host cores.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = [os.path.join(_HERE, "aba_oracle.c"), os.path.join(_HERE, "pgs_oracle.c")]
DEPS = SOURCES + [os.path.join(_HERE, "aba_fwd.inc"), os.path.join(_HERE, "oracle.h")]
# joint types (oracle.h)
ORC_REVOLUTE, ORC_FREE, ORC_PRISMATIC, ORC_SPHERICAL = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (portable -O2, no host-specific ISA)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp,
                               *SOURCES, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


NATIVE_LIB_PATH = os.path.join(_HERE, "liboracle_native.so")


def build_native() -> str:
    """The same oracle sources optimised for the host it is built on (-O3
    -march=native), for timing the CPU baseline; FP contraction stays off so
    that its arithmetic rounds as the portable build's does."""
    tmp = NATIVE_LIB_PATH + f".{os.getpid()}.tmp"
    subprocess.check_call(["gcc", "-O3", "-march=native", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared",
                           "-o", tmp, *SOURCES, "-lm"])
    os.replace(tmp, NATIVE_LIB_PATH)
    return NATIVE_LIB_PATH


_lib = None


def _configure(L):
    P = ctypes.c_void_p
    for name in ("orc_nq", "orc_nv", "orc_nu"):
        getattr(L, name).restype = ctypes.c_int
        getattr(L, name).argtypes = [P]
    L.orc_fd.argtypes = [P, P, P, P, P]
    L.orc_fd_c.argtypes = [P, P, P, P, P]
    L.orc_fd_vjp.argtypes = [P, P, P, P, P, P, P, P]
    L.orc_step.argtypes = [P, P, P, P, ctypes.c_double, P, P]
    L.orc_rollout.argtypes = [P, P, P, P, ctypes.c_double, ctypes.c_int, P, P, P]
    L.orc_rollout.restype = ctypes.c_int
    L.orc_rollout_c.argtypes = [P, P, P, P, ctypes.c_double, ctypes.c_int, P, P]
    L.orc_rollout_c.restype = ctypes.c_int
    L.orc_rollout_grad.argtypes = [P, P, P, P, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int, P, P, P, P, P, P, P, P]
    L.orc_rollout_grad.restype = ctypes.c_int
    L.orc_adjoint_along.argtypes = [P, P, P, ctypes.c_double, ctypes.c_int, P, P, P, P, P, P]
    L.orc_adjoint_along.restype = ctypes.c_int
    L.orc_rollout_grad_params.argtypes = [P, P, P, P, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_int, P, P, P, P, P, P, P, P, P, P]
    L.orc_rollout_grad_params.restype = ctypes.c_int
    L.orc_adjoint_along_params.argtypes = [P, P, P, ctypes.c_double, ctypes.c_int, P, P, P, P, P, P, P, P]
    L.orc_adjoint_along_params.restype = ctypes.c_int
    I = ctypes.c_int
    L.orc_pgs_solve.argtypes = [I, I, P, P, P, P, P, P, P]
    L.orc_pgs_solve.restype = None
    L.orc_pgs_solve_c.argtypes = [I, I, P, P, P, P, P, P]
    L.orc_pgs_solve_c.restype = None
    L.orc_pgs_adjoint.argtypes = [I, I, P, P, P, P, P, P, P, P, P, P, P]
    L.orc_pgs_adjoint.restype = None
    D = ctypes.c_double
    L.orc_contact_assembly.argtypes = [P, P, P, P, P, P, P]
    L.orc_contact_assembly.restype = I
    L.orc_step_contact.argtypes = [P, P, P, P, P, D, P, P, P]
    L.orc_step_contact.restype = I
    L.orc_step_contact_c.argtypes = [P, P, P, P, P, D, P, P]
    L.orc_step_contact_c.restype = I
    L.orc_rollout_contact.argtypes = [P, P, P, P, P, D, I, P, P, P, P]
    L.orc_rollout_contact.restype = I
    L.orc_rollout_contact_grad.argtypes = [P, P, P, P, P, D, I, P, P, P, P, P, P]
    L.orc_rollout_contact_grad.restype = I
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        _lib = _configure(ctypes.CDLL(LIB_PATH))
    return _lib


class use_library:
    """Context manager: route every oracle call through another build of the
    oracle (used by the mutation tests to check that the pins catch planted
    mistakes)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = _configure(ctypes.CDLL(self.path))
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


class _CModel(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int),
                ("parent", ctypes.c_void_p), ("jtype", ctypes.c_void_p),
                ("E_T", ctypes.c_void_p), ("r_T", ctypes.c_void_p),
                ("axis", ctypes.c_void_p), ("mass", ctypes.c_void_p),
                ("com", ctypes.c_void_p), ("Ic", ctypes.c_void_p),
                ("gravity", ctypes.c_void_p), ("limits", ctypes.c_void_p)]


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Model:
    """An articulated system prepared for the oracle (FP64 copies)."""

    def __init__(self, system, gravity=(0.0, -9.81, 0.0)):
        f = lambda x: np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        self.parent = np.ascontiguousarray(np.asarray(system.parent, dtype=np.int32))
        self.jtype = np.ascontiguousarray(np.asarray(system.jtype, dtype=np.int32))
        self.E_T = f(system.E_T).reshape(-1)
        self.r_T = f(system.r_T).reshape(-1)
        # a joint axis is a direction: the joint rotates about a / |a|
        # (a spherical joint has none; its entry is not read)
        ax = f(system.axis).reshape(-1, 3)
        nrm = np.linalg.norm(ax, axis=1, keepdims=True)
        self.axis = np.ascontiguousarray(np.where(nrm > 0, ax / np.where(nrm > 0, nrm, 1.0), 0.0).reshape(-1))
        self.mass = f(system.mass).reshape(-1)
        self.com = f(system.com).reshape(-1)
        self.Ic = f(system.Ic).reshape(-1)
        self.gravity = f(gravity).reshape(3)
        # optional joint limits [n, 4]: lo, hi, stiffness, damping
        lim = getattr(system, "limits", None)
        self.limits = None if lim is None else f(lim).reshape(-1)
        self.c = _CModel(int(self.parent.shape[0]), _p(self.parent), _p(self.jtype),
                         _p(self.E_T), _p(self.r_T), _p(self.axis), _p(self.mass),
                         _p(self.com), _p(self.Ic), _p(self.gravity),
                         _p(self.limits) if self.limits is not None else None)
        self.ref = ctypes.byref(self.c)
        L = lib()
        self.nq, self.nv, self.nu = L.orc_nq(self.ref), L.orc_nv(self.ref), L.orc_nu(self.ref)
        self.n = int(self.parent.shape[0])


def _f64(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


def _c128(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


def fd(m: Model, q, qd, tau):
    """Forward dynamics qdd = FD(q, qd, tau)."""
    q, qd, tau = _f64(q, m.nq), _f64(qd, m.nv), _f64(tau, m.nu)
    out = np.zeros(m.nv)
    lib().orc_fd(m.ref, _p(q), _p(qd), _p(tau), _p(out))
    return out


def fd_complex(m: Model, q, qd, tau):
    q, qd, tau = _c128(q, m.nq), _c128(qd, m.nv), _c128(tau, m.nu)
    out = np.zeros(m.nv, dtype=np.complex128)
    lib().orc_fd_c(m.ref, _p(q), _p(qd), _p(tau), _p(out))
    return out


def fd_vjp(m: Model, q, qd, tau, qdd_bar):
    """Reverse mode of one forward-dynamics evaluation."""
    q, qd, tau, qb = _f64(q, m.nq), _f64(qd, m.nv), _f64(tau, m.nu), _f64(qdd_bar, m.nv)
    gq, gqd, gt = np.zeros(m.nq), np.zeros(m.nv), np.zeros(m.nu)
    lib().orc_fd_vjp(m.ref, _p(q), _p(qd), _p(tau), _p(qb), _p(gq), _p(gqd), _p(gt))
    return gq, gqd, gt


def step(m: Model, q, qd, tau, dt):
    q, qd, tau = _f64(q, m.nq), _f64(qd, m.nv), _f64(tau, m.nu)
    q1, qd1 = np.zeros(m.nq), np.zeros(m.nv)
    lib().orc_step(m.ref, _p(q), _p(qd), _p(tau), float(dt), _p(q1), _p(qd1))
    return q1, qd1


def rollout(m: Model, q0, qd0, tau, dt, traj: bool = False):
    """T-step rollout; tau is [T, nu].  Returns qT, qdT (and traj [T, nq+nv])."""
    tau = _f64(tau)
    T = int(tau.shape[0])
    tau = tau.reshape(T, m.nu)
    q0, qd0 = _f64(q0, m.nq), _f64(qd0, m.nv)
    qT, qdT = np.zeros(m.nq), np.zeros(m.nv)
    tr = np.zeros((T, m.nq + m.nv)) if traj else None
    rc = lib().orc_rollout(m.ref, _p(q0), _p(qd0), _p(np.ascontiguousarray(tau)), float(dt), T,
                           _p(qT), _p(qdT), _p(tr) if traj else None)
    if rc != 0:
        raise RuntimeError("oracle rollout failed")
    return (qT, qdT, tr) if traj else (qT, qdT)


def rollout_complex(m: Model, q0, qd0, tau, dt):
    tau = _c128(tau)
    T = int(tau.shape[0])
    tau = tau.reshape(T, m.nu)
    q0, qd0 = _c128(q0, m.nq), _c128(qd0, m.nv)
    qT, qdT = np.zeros(m.nq, dtype=np.complex128), np.zeros(m.nv, dtype=np.complex128)
    rc = lib().orc_rollout_c(m.ref, _p(q0), _p(qd0), _p(np.ascontiguousarray(tau)), float(dt),
                             T, _p(qT), _p(qdT))
    if rc != 0:
        raise RuntimeError("oracle complex rollout failed")
    return qT, qdT


def rollout_grad(m: Model, q0, qd0, tau, dt, gqT, gqdT, gtraj=None, K: int = 1):
    """Adjoint-method gradient of <gqT, q^T> + <gqdT, qd^T> + <gtraj, traj>
    with respect to (q0, qd0, tau).  K >= 1: checkpoint every K steps;
    K == 0: store every step's intermediates.  Returns gq0, gqd0, gtau, qT, qdT."""
    tau = _f64(tau)
    T = int(tau.shape[0])
    tau = np.ascontiguousarray(tau.reshape(T, m.nu))
    q0, qd0 = _f64(q0, m.nq), _f64(qd0, m.nv)
    gqT, gqdT = _f64(gqT, m.nq), _f64(gqdT, m.nv)
    gtr = None if gtraj is None else np.ascontiguousarray(_f64(gtraj).reshape(T, m.nq + m.nv))
    gq0, gqd0, gtau = np.zeros(m.nq), np.zeros(m.nv), np.zeros((T, m.nu))
    qT, qdT = np.zeros(m.nq), np.zeros(m.nv)
    rc = lib().orc_rollout_grad(m.ref, _p(q0), _p(qd0), _p(tau), float(dt), T, int(K),
                                _p(gqT), _p(gqdT), _p(gtr) if gtr is not None else None,
                                _p(gq0), _p(gqd0), _p(gtau), _p(qT), _p(qdT))
    if rc != 0:
        raise RuntimeError("oracle rollout_grad failed")
    return gq0, gqd0, gtau, qT, qdT


def rollout_grad_params(m: Model, q0, qd0, tau, dt, gqT, gqdT, gtraj=None, K: int = 1):
    """As rollout_grad, plus gradients with respect to model parameters,
    summed over the rollout.  Returns gq0, gqd0, gtau, gparam [n, 10],
    gframe [n, 9], qT, qdT.  gparam: every link's ten inertial parameters
    (m, h = m c, I about the link origin: xx yy zz xy xz yz; link frame).
    gframe: every 1-dof link's placement and axis (phi_bar, r_T_bar,
    axis_bar; zero for a free root), as orc_rollout_grad_params states."""
    tau = _f64(tau)
    T = int(tau.shape[0])
    tau = np.ascontiguousarray(tau.reshape(T, m.nu))
    q0, qd0 = _f64(q0, m.nq), _f64(qd0, m.nv)
    gqT, gqdT = _f64(gqT, m.nq), _f64(gqdT, m.nv)
    gtr = None if gtraj is None else np.ascontiguousarray(_f64(gtraj).reshape(T, m.nq + m.nv))
    gq0, gqd0, gtau = np.zeros(m.nq), np.zeros(m.nv), np.zeros((T, m.nu))
    gparam, gframe = np.zeros((m.n, 10)), np.zeros((m.n, 9))
    qT, qdT = np.zeros(m.nq), np.zeros(m.nv)
    rc = lib().orc_rollout_grad_params(m.ref, _p(q0), _p(qd0), _p(tau), float(dt), T, int(K),
                                       _p(gqT), _p(gqdT), _p(gtr) if gtr is not None else None,
                                       _p(gq0), _p(gqd0), _p(gtau), _p(gparam), _p(gframe), _p(qT), _p(qdT))
    if rc != 0:
        raise RuntimeError("oracle rollout_grad_params failed")
    return gq0, gqd0, gtau, gparam, gframe, qT, qdT


def adjoint_along_params(m: Model, states, tau, dt, gqT, gqdT, gtraj=None):
    """adjoint_along plus the parameter gradients gparam [n, 10] and
    gframe [n, 9] (see rollout_grad_params)."""
    tau = _f64(tau)
    T = int(tau.shape[0])
    tau = np.ascontiguousarray(tau.reshape(T, m.nu))
    st = np.ascontiguousarray(_f64(states).reshape(T, m.nq + m.nv))
    gqT, gqdT = _f64(gqT, m.nq), _f64(gqdT, m.nv)
    gtr = None if gtraj is None else np.ascontiguousarray(_f64(gtraj).reshape(T, m.nq + m.nv))
    gq0, gqd0, gtau = np.zeros(m.nq), np.zeros(m.nv), np.zeros((T, m.nu))
    gparam, gframe = np.zeros((m.n, 10)), np.zeros((m.n, 9))
    rc = lib().orc_adjoint_along_params(m.ref, _p(st), _p(tau), float(dt), T, _p(gqT), _p(gqdT),
                                        _p(gtr) if gtr is not None else None, _p(gq0), _p(gqd0),
                                        _p(gtau), _p(gparam), _p(gframe))
    if rc != 0:
        raise RuntimeError("oracle adjoint_along_params failed")
    return gq0, gqd0, gtau, gparam, gframe


def adjoint_along(m: Model, states, tau, dt, gqT, gqdT, gtraj=None):
    """Reverse sweep along a given trajectory: states [T, nq+nv] holds the
    initial state of every step (x^0 .. x^{T-1}).  Returns gq0, gqd0, gtau."""
    tau = _f64(tau)
    T = int(tau.shape[0])
    tau = np.ascontiguousarray(tau.reshape(T, m.nu))
    st = np.ascontiguousarray(_f64(states).reshape(T, m.nq + m.nv))
    gqT, gqdT = _f64(gqT, m.nq), _f64(gqdT, m.nv)
    gtr = None if gtraj is None else np.ascontiguousarray(_f64(gtraj).reshape(T, m.nq + m.nv))
    gq0, gqd0, gtau = np.zeros(m.nq), np.zeros(m.nv), np.zeros((T, m.nu))
    rc = lib().orc_adjoint_along(m.ref, _p(st), _p(tau), float(dt), T, _p(gqT), _p(gqdT),
                                 _p(gtr) if gtr is not None else None, _p(gq0), _p(gqd0), _p(gtau))
    if rc != 0:
        raise RuntimeError("oracle adjoint_along failed")
    return gq0, gqd0, gtau


def ball_tangent(system, q, gq):
    """gq with the radial part of every spherical joint's quaternion adjoint
    removed: g - (g . qh) qh, qh = q / |q|, i.e. the gradient along the unit
    sphere.  On the sphere the step map is the same for every continuation
    of R(quat) off it, so only this part is defined by the joint model (our
    reading: a ball joint's state is a unit quaternion, Sec. 2 and App. G;
    the integrator renormalises it every step).  q, gq: one system's [nq]
    (or [..., nq]) arrays."""
    g = np.array(gq, dtype=np.float64, copy=True)
    qi = 0
    for i in range(system.n):
        jt = int(system.jtype[i])
        if jt == ORC_SPHERICAL:
            qh = np.asarray(q[..., qi:qi + 4], dtype=np.float64)
            qh = qh / np.linalg.norm(qh, axis=-1, keepdims=True)
            gi = g[..., qi:qi + 4]
            g[..., qi:qi + 4] = gi - np.sum(gi * qh, axis=-1, keepdims=True) * qh
        qi += 7 if jt == ORC_FREE else 4 if jt == ORC_SPHERICAL else 1
    return g


def map_threads(fn, items, threads: int | None = None):
    """Run fn over items on a thread pool (the C calls release the GIL)."""
    threads = threads or min(16, os.cpu_count() or 1)
    if threads <= 1:
        return [fn(x) for x in items]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, items))


# ---------------------------------------------------------------- contact solver

def _vec(x, n, dtype=np.float64):
    return np.ascontiguousarray(np.asarray(x, dtype=dtype).reshape(n))


def pgs_solve(A, b, lo, hi, x0, niter, sweeps=False):
    """Projected Gauss-Seidel on a = A x + b, lo <= x <= hi (one problem,
    A [n, n]).  Returns x, or (x, sweeps [niter + 1, n]) with the vector at
    the start of every sweep and the result."""
    n = int(np.asarray(b).size)
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64).reshape(n, n))
    b, lo, hi, x0 = (_vec(v, n) for v in (b, lo, hi, x0))
    x = np.zeros(n)
    sw = np.zeros((niter + 1, n)) if sweeps else None
    lib().orc_pgs_solve(n, int(niter), _p(A), _p(b), _p(lo), _p(hi), _p(x0), _p(x),
                        _p(sw) if sweeps else None)
    return (x, sw) if sweeps else x


def pgs_solve_complex(A, b, lo, hi, x0, niter):
    """pgs_solve in complex arithmetic (complex-step checks)."""
    n = int(np.asarray(b).size)
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128).reshape(n, n))
    b, lo, hi, x0 = (_vec(v, n, np.complex128) for v in (b, lo, hi, x0))
    x = np.zeros(n, np.complex128)
    lib().orc_pgs_solve_c(n, int(niter), _p(A), _p(b), _p(lo), _p(hi), _p(x0), _p(x))
    return x


def pgs_adjoint(A, b, lo, hi, sweeps, xbar):
    """Reverse of pgs_solve from its stored sweeps: returns A_bar [n, n],
    b_bar, lo_bar, hi_bar, x0_bar."""
    n = int(np.asarray(b).size)
    niter = int(np.asarray(sweeps).shape[0]) - 1
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64).reshape(n, n))
    b, lo, hi, xbar = (_vec(v, n) for v in (b, lo, hi, xbar))
    sw = np.ascontiguousarray(np.asarray(sweeps, dtype=np.float64).reshape(niter + 1, n))
    Ab, bb, lb, hb, x0b = np.zeros((n, n)), np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_pgs_adjoint(n, niter, _p(A), _p(b), _p(lo), _p(hi), _p(sw), _p(xbar), _p(Ab), _p(bb), _p(lb),
                          _p(hb), _p(x0b))
    return Ab, bb, lb, hb, x0b


# ---------------------------------------------------------------- contact in the step

class _CContacts(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("link", ctypes.c_void_p), ("center", ctypes.c_void_p),
                ("radius", ctypes.c_void_p), ("mu", ctypes.c_double), ("beta", ctypes.c_double),
                ("niter", ctypes.c_int)]


class Contacts:
    """Contact spheres against the ground plane y = 0 (contact.inc): per
    sphere its link, centre (link coordinates) and radius; box friction mu,
    Baumgarte factor beta, PGS sweeps niter per solve."""

    def __init__(self, link, center, radius, mu=0.5, beta=0.0, niter=50):
        self.link = np.ascontiguousarray(np.asarray(link, dtype=np.int32).reshape(-1))
        self.n = int(self.link.size)
        self.center = np.ascontiguousarray(np.asarray(center, dtype=np.float64).reshape(self.n, 3))
        self.radius = np.ascontiguousarray(np.asarray(radius, dtype=np.float64).reshape(self.n))
        self.c = _CContacts(self.n, _p(self.link), _p(self.center), _p(self.radius), float(mu), float(beta),
                            int(niter))
        self.ref = ctypes.byref(self.c)


def contact_assembly(m: Model, C: Contacts, q):
    """Active contacts, gaps, J [3m, nv] and M^-1 J^T [nv, 3m] at q."""
    q = _f64(q, m.nq)
    cap = max(C.n, 1)
    act, phi = np.zeros(cap, np.int32), np.zeros(cap)
    J, MJ = np.zeros(3 * cap * m.nv), np.zeros(3 * cap * m.nv)
    na = lib().orc_contact_assembly(m.ref, C.ref, _p(q), _p(act), _p(phi), _p(J), _p(MJ))
    return act[:na], phi[:na], J[:3 * na * m.nv].reshape(3 * na, m.nv), MJ[:3 * na * m.nv].reshape(m.nv, 3 * na)


def step_contact(m: Model, C: Contacts, q, qd, tau, dt):
    """One step with contact: returns q1, qd1, the active-contact count and
    their impulses [3m] (normal, tangent x, tangent z per contact)."""
    q, qd, tau = _f64(q, m.nq), _f64(qd, m.nv), _f64(tau, m.nu)
    q1, qd1, lam = np.zeros(m.nq), np.zeros(m.nv), np.zeros(3 * max(C.n, 1))
    na = lib().orc_step_contact(m.ref, C.ref, _p(q), _p(qd), _p(tau), float(dt), _p(q1), _p(qd1), _p(lam))
    return q1, qd1, na, lam[:3 * na]


def step_contact_complex(m: Model, C: Contacts, q, qd, tau, dt):
    q, qd, tau = _c128(q, m.nq), _c128(qd, m.nv), _c128(tau, m.nu)
    q1, qd1 = np.zeros(m.nq, np.complex128), np.zeros(m.nv, np.complex128)
    lib().orc_step_contact_c(m.ref, C.ref, _p(q), _p(qd), _p(tau), float(dt), _p(q1), _p(qd1))
    return q1, qd1


def rollout_contact(m: Model, C: Contacts, q0, qd0, tau, dt, traj: bool = False):
    """Rollout with contact; returns qT, qdT, the per-step active-contact
    counts, and with traj=True the states x^{t+1} [T, nq+nv]."""
    tau = np.ascontiguousarray(np.asarray(tau, dtype=np.float64).reshape(-1, m.nu) if m.nu else
                               np.zeros((np.asarray(tau).shape[0], 0)))
    T = tau.shape[0]
    q0, qd0 = _f64(q0, m.nq), _f64(qd0, m.nv)
    qT, qdT, nc = np.zeros(m.nq), np.zeros(m.nv), np.zeros(T, np.int32)
    tr = np.zeros((T, m.nq + m.nv)) if traj else None
    rc = lib().orc_rollout_contact(m.ref, C.ref, _p(q0), _p(qd0), _p(tau), float(dt), T, _p(qT), _p(qdT),
                                   _p(tr) if traj else None, _p(nc))
    if rc != 0:
        raise RuntimeError("orc_rollout_contact failed")
    return (qT, qdT, nc, tr) if traj else (qT, qdT, nc)


def rollout_contact_grad(m: Model, C: Contacts, q0, qd0, tau, dt, gqT, gqdT, mu_grad: bool = False):
    """Gradient of <gqT, qT> + <gqdT, qdT> through a rollout with contact:
    returns gq0, gqd0, gtau [T, nu], and with mu_grad the derivative with
    respect to the friction coefficient."""
    tau = np.ascontiguousarray(np.asarray(tau, dtype=np.float64).reshape(-1, m.nu) if m.nu else
                               np.zeros((np.asarray(tau).shape[0], 0)))
    T = tau.shape[0]
    q0, qd0, gqT, gqdT = _f64(q0, m.nq), _f64(qd0, m.nv), _f64(gqT, m.nq), _f64(gqdT, m.nv)
    gq0, gqd0, gtau = np.zeros(m.nq), np.zeros(m.nv), np.zeros((T, m.nu))
    gmu = ctypes.c_double()
    rc = lib().orc_rollout_contact_grad(m.ref, C.ref, _p(q0), _p(qd0), _p(tau), float(dt), T, _p(gqT), _p(gqdT),
                                        _p(gq0), _p(gqd0), _p(gtau),
                                        ctypes.byref(gmu) if mu_grad else None)
    if rc != 0:
        raise RuntimeError("orc_rollout_contact_grad failed")
    return (gq0, gqd0, gtau, gmu.value) if mu_grad else (gq0, gqd0, gtau)
