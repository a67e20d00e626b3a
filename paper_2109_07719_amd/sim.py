"""Python front end of the C ABI: a batch handle and a differentiable rollout.

PyTorch supplies device memory and the stream; all arithmetic of the
forward rollout, the adjoint pass and single forward-dynamics evaluations
runs in the HIP kernels behind ``include/abadj.h``.

  sim = Sim(systems, gravity, dtype=torch.float32)
  qT, qdT = rollout(sim, q0, qd0, tau, dt, K=1)          # differentiable
  qdd = sim.aba(q, qd, tau)                              # forward dynamics

Method: ABA forward dynamics (Sec. 3), semi-implicit Euler, adjoint method
through time (Sec. 3, Eq. adj_back; Sec. 4.1, Eq. adj_r) with the initial
state of each step checkpointed and the step recomputed in the backward pass
(Sec. 4.2, Eq. intermediate), checkpoint interval K (App. B).
"""
from __future__ import annotations

import ctypes
import weakref

import numpy as np
import torch

from . import _native as N


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Sim:
    """A batch of articulated systems packed for the GPU.

    systems: sequence of objects with numpy attributes parent, jtype, E_T
    (n,3,3), r_T (n,3), axis (n,3), mass (n,), com (n,3), Ic (n,6); links in
    topological order.  The handle's dtype (float32 or float64) is the
    arithmetic type of every kernel.
    """

    def __init__(self, systems, gravity=(0.0, -9.81, 0.0), dtype=torch.float32,
                 device="cuda"):
        L = N.lib()
        self.dtype = dtype
        self.device = torch.device(device)
        if dtype not in (torch.float32, torch.float64):
            raise TypeError("dtype must be torch.float32 or torch.float64")
        cat = lambda name, shape: np.ascontiguousarray(
            np.concatenate([np.asarray(getattr(s, name), dtype=np.float64).reshape(-1, *shape)
                            for s in systems]).reshape(-1))
        self._parent = np.ascontiguousarray(np.concatenate(
            [np.asarray(s.parent, dtype=np.int32) for s in systems]))
        self._jtype = np.ascontiguousarray(np.concatenate(
            [np.asarray(s.jtype, dtype=np.int32) for s in systems]))
        sizes = [len(s.parent) for s in systems]
        self._off = np.ascontiguousarray(np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32))
        self._E_T = cat("E_T", (9,))
        self._r_T = cat("r_T", (3,))
        self._axis = cat("axis", (3,))
        self._mass = cat("mass", ())
        self._com = cat("com", (3,))
        self._Ic = cat("Ic", (6,))
        self._g = np.ascontiguousarray(np.asarray(gravity, dtype=np.float64).reshape(3))
        # optional joint limits [n, 4] per system (lo, hi, stiffness, damping)
        if any(getattr(s, "limits", None) is not None for s in systems):
            none = lambda s: np.tile([-1e30, 1e30, 0.0, 0.0], (len(s.parent), 1))
            self._lim = np.ascontiguousarray(np.concatenate(
                [np.asarray(s.limits if getattr(s, "limits", None) is not None else none(s),
                            dtype=np.float64).reshape(-1, 4) for s in systems]).reshape(-1))
        else:
            self._lim = None
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        topo = N.SimTopology(len(systems), p(self._off), p(self._parent), p(self._jtype))
        prm = N.SimParams(p(self._E_T), p(self._r_T), p(self._axis), p(self._mass), p(self._com),
                          p(self._Ic), p(self._g), p(self._lim) if self._lim is not None else None)
        h = ctypes.c_void_p()
        N.check(L.sim_create(ctypes.byref(topo), ctypes.byref(prm),
                             N.SIM_F64 if dtype == torch.float64 else N.SIM_F32, ctypes.byref(h)))
        self._h = h
        # released when the object is collected, or at interpreter exit while
        # the ctypes library is still loaded
        self._release = weakref.finalize(self, L.sim_destroy, h)
        info = N.SimInfo()
        N.check(L.sim_get_info(h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in N.SimInfo._fields_}
        self.nq, self.nv, self.nu = info.nq, info.nv, info.nu

    @property
    def adjoint_dtype(self):
        """Arithmetic of the backward pass: each step's recompute and reverse
        passes (torch.float64 by default; an FP32 handle may select
        torch.float32)."""
        return torch.float64 if self.info["adjoint_dtype"] == N.SIM_F64 else torch.float32

    def set_adjoint_dtype(self, dtype) -> None:
        """FP32 handles: run the backward pass's per-step recompute and
        reverse passes in FP64 (default; inputs, outputs, checkpoints and
        the forward stay FP32) or in FP32."""
        if dtype not in (torch.float32, torch.float64):
            raise TypeError("dtype must be torch.float32 or torch.float64")
        N.check(N.lib().sim_set_adjoint_dtype(self._h, N.SIM_F64 if dtype == torch.float64 else N.SIM_F32))
        self.info["adjoint_dtype"] = N.SIM_F64 if dtype == torch.float64 else N.SIM_F32

    def close(self):
        """Release the handle now (also done when the object is collected)."""
        release = getattr(self, "_release", None)
        if release is not None:
            release()
            self._h = ctypes.c_void_p()   # later calls see a null handle and fail cleanly

    # ------------------------------------------------------------------ checks
    def _t(self, x, n, name, allow_none=False):
        if x is None:
            if allow_none:
                return None
            raise ValueError(f"{name} is required")
        if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA tensor")
        if x.dtype != self.dtype:
            raise TypeError(f"{name} must have dtype {self.dtype}")
        if not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if x.numel() != n:
            raise ValueError(f"{name} has {x.numel()} elements, expected {n}")
        return x

    def status(self) -> int:
        """Non-finite numbers written to outputs since the last call (resets
        the counter; synchronises the current stream)."""
        n = ctypes.c_int()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        N.check(N.lib().sim_status(self._h, ctypes.c_void_p(stream), ctypes.byref(n)))
        return int(n.value)

    @property
    def tiling(self) -> dict:
        """Launch geometry: waves_per_block, pairs_per_block, pipelined."""
        t = N.SimTiling()
        N.check(N.lib().sim_get_tiling(self._h, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in N.SimTiling._fields_}

    def set_tiling(self, waves_per_block: int = 1, pairs_per_block: int = 1, pipelined: bool = True) -> None:
        t = N.SimTiling(int(waves_per_block), int(pairs_per_block), int(bool(pipelined)))
        N.check(N.lib().sim_set_tiling(self._h, ctypes.byref(t)))

    def autotune(self, K: int = 1, T_probe: int = 200) -> dict:
        """Time every launch geometry on probe rollouts and keep the fastest
        (sim_autotune); returns the chosen tiling and its ms per probe step."""
        t, ms = N.SimTiling(), ctypes.c_double()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        N.check(N.lib().sim_autotune(self._h, int(K), int(T_probe), ctypes.c_void_p(stream), ctypes.byref(t),
                                     ctypes.byref(ms)))
        out = {f: getattr(t, f) for f, _ in N.SimTiling._fields_}
        out["ms_per_probe_step"] = ms.value
        return out

    def workspace_bytes(self, T: int, K: int = 1) -> int:
        b = ctypes.c_size_t()
        N.check(N.lib().sim_workspace_bytes(self._h, int(T), int(K), ctypes.byref(b)))
        return int(b.value)

    def new_workspace(self, T: int, K: int = 1):
        return torch.empty(max(self.workspace_bytes(T, K), 1), dtype=torch.uint8, device=self.device)

    def flops(self, kind: int) -> float:
        f = ctypes.c_double()
        N.check(N.lib().sim_flops(self._h, int(kind), ctypes.byref(f)))
        return float(f.value)

    # ------------------------------------------------------------------ calls
    def aba(self, q, qd, tau, out=None):
        """Forward dynamics qdd = FD(q, qd, tau) for every system."""
        self._t(q, self.nq, "q"), self._t(qd, self.nv, "qd"), self._t(tau, self.nu, "tau")
        qdd = out if out is not None else torch.empty(self.nv, dtype=self.dtype, device=q.device)
        N.check(N.lib().sim_aba(self._h, _ptr(q), _ptr(qd), _ptr(tau), _ptr(qdd), _stream()))
        return qdd

    def forward(self, q0, qd0, tau, dt, K=1, workspace=None, traj=False, out=None):
        """Rollout of T = tau.shape[0] steps.  workspace=None: plain forward
        (no checkpoints).  Returns (qT, qdT, traj or None)."""
        tau = tau.reshape(-1, self.nu) if self.nu else tau
        T = int(tau.shape[0])
        self._t(q0, self.nq, "q0"), self._t(qd0, self.nv, "qd0"), self._t(tau, T * self.nu, "tau")
        dev = q0.device
        if out is None:
            qT = torch.empty(self.nq, dtype=self.dtype, device=dev)
            qdT = torch.empty(self.nv, dtype=self.dtype, device=dev)
            tr = torch.empty((T, self.nq + self.nv), dtype=self.dtype, device=dev) if traj else None
        else:
            qT, qdT, tr = out
        wsb = workspace.numel() if workspace is not None else 0
        N.check(N.lib().sim_forward(self._h, _ptr(q0), _ptr(qd0), _ptr(tau), float(dt), T, int(K),
                                    _ptr(qT), _ptr(qdT), _ptr(tr), _ptr(workspace), wsb, _stream()))
        return qT, qdT, tr

    def forward_jvp(self, q0, qd0, tau, dq0, dqd0, dtau, dt, traj=False):
        """Forward-mode rollout along the input direction (dq0, dqd0, dtau).
        Returns (qT, qdT, dqT, dqdT) and, with traj=True, also (traj, dtraj)."""
        tau = tau.reshape(-1, self.nu) if self.nu else tau
        T = int(tau.shape[0])
        self._t(q0, self.nq, "q0"), self._t(qd0, self.nv, "qd0"), self._t(tau, T * self.nu, "tau")
        self._t(dq0, self.nq, "dq0"), self._t(dqd0, self.nv, "dqd0")
        self._t(dtau.reshape(-1), T * self.nu, "dtau")
        e = lambda *shape: torch.empty(shape, dtype=self.dtype, device=q0.device)
        qT, qdT, dqT, dqdT = e(self.nq), e(self.nv), e(self.nq), e(self.nv)
        tr, dtr = (e(T, self.nq + self.nv), e(T, self.nq + self.nv)) if traj else (None, None)
        N.check(N.lib().sim_forward_jvp(self._h, _ptr(q0), _ptr(qd0), _ptr(tau), _ptr(dq0), _ptr(dqd0),
                                        _ptr(dtau), float(dt), T, _ptr(qT), _ptr(qdT), _ptr(dqT), _ptr(dqdT),
                                        _ptr(tr), _ptr(dtr), _stream()))
        return (qT, qdT, dqT, dqdT, tr, dtr) if traj else (qT, qdT, dqT, dqdT)

    def backward(self, tau, dt, K, workspace, gqT, gqdT, gtraj=None, out=None, params=False):
        """Adjoint pass after forward() on the same workspace.  Returns
        (gq0, gqd0, gtau), and with params=True also, summed over the
        rollout, the gradient with respect to every link's ten inertial
        parameters [n_links, 10] (m, h = m c, I about the link origin xx yy
        zz xy xz yz; caller's link frames) and with respect to every 1-dof
        link's placement and axis [n_links, 9] (phi_bar: rotation of the
        joint frame E_T -> exp(-[phi]x) E_T; r_T_bar; axis_bar along the unit
        sphere; zeros for a free root)."""
        tau = tau.reshape(-1, self.nu) if self.nu else tau
        T = int(tau.shape[0])
        self._t(gqT, self.nq, "gqT"), self._t(gqdT, self.nv, "gqdT")
        self._t(gtraj, T * (self.nq + self.nv), "gtraj", allow_none=True)
        dev = gqT.device
        if out is None:
            gq0 = torch.empty(self.nq, dtype=self.dtype, device=dev)
            gqd0 = torch.empty(self.nv, dtype=self.dtype, device=dev)
            gtau = torch.empty((T, self.nu), dtype=self.dtype, device=dev)
            gparam = torch.empty((self.info["n_links"], 10), dtype=self.dtype, device=dev) if params else None
            gframe = torch.empty((self.info["n_links"], 9), dtype=self.dtype, device=dev) if params else None
        else:
            gq0, gqd0, gtau = out[:3]
            gparam, gframe = (out[3], out[4]) if params else (None, None)
        N.check(N.lib().sim_backward(self._h, _ptr(tau), float(dt), T, int(K), _ptr(gqT), _ptr(gqdT),
                                     _ptr(gtraj), _ptr(gq0), _ptr(gqd0), _ptr(gtau), _ptr(gparam), _ptr(gframe),
                                     _ptr(workspace), workspace.numel(), _stream()))
        return (gq0, gqd0, gtau, gparam, gframe) if params else (gq0, gqd0, gtau)


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim, q0, qd0, tau, dt, K, want_traj):
        q0, qd0, tau = q0.contiguous(), qd0.contiguous(), tau.contiguous()
        T = int(tau.shape[0])
        ws = sim.new_workspace(T, K)
        qT, qdT, tr = sim.forward(q0, qd0, tau, dt, K=K, workspace=ws, traj=want_traj)
        ctx.sim, ctx.dt, ctx.K, ctx.want_traj = sim, dt, K, want_traj
        ctx.save_for_backward(tau, ws)
        if want_traj:
            return qT, qdT, tr
        return qT, qdT

    @staticmethod
    def backward(ctx, *grads):
        tau, ws = ctx.saved_tensors
        sim = ctx.sim
        gqT, gqdT = grads[0], grads[1]
        gtraj = grads[2] if ctx.want_traj else None
        z = lambda n: torch.zeros(n, dtype=sim.dtype, device=tau.device)
        gqT = z(sim.nq) if gqT is None else gqT.contiguous()
        gqdT = z(sim.nv) if gqdT is None else gqdT.contiguous()
        if gtraj is not None:
            gtraj = gtraj.contiguous()
        gq0, gqd0, gtau = sim.backward(tau, ctx.dt, ctx.K, ws, gqT, gqdT, gtraj)
        return None, gq0, gqd0, gtau.reshape(tau.shape), None, None, None


def rollout(sim: Sim, q0, qd0, tau, dt: float, K: int = 1, traj: bool = False):
    """Differentiable T-step rollout (T = tau.shape[0]); gradients flow to
    q0, qd0 and tau through the adjoint kernel.  Returns (qT, qdT) or
    (qT, qdT, traj)."""
    return _Rollout.apply(sim, q0, qd0, tau, float(dt), int(K), bool(traj))
