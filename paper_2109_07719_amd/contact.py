"""Rollouts with contact inside the step on the GPU and their gradient
(Sec. 4.1 "Collision resolution": detection, the MLCP of Eq. mlcp by
projected Gauss-Seidel, velocity impulses), through the C ABI
(`sim_contact_rollout`, `sim_contact_rollout_grad` in include/abadj.h).

A batch shares one topology and one set of contact spheres (links); every
system has its own inertial, placement and sphere parameters.  Arrays are
entry-major, as at the C ABI: q [nq][B], qd [nv][B], tau [T][nu][B], the
trajectory [T + 1][nq + nv][B].  Argument marshalling only: every step runs
in the library's kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _native as N

_DT = {torch.float32: N.SIM_F32, torch.float64: N.SIM_F64}


class _Tiling(ctypes.Structure):
    _fields_ = [("rollout_systems_per_wave", ctypes.c_int), ("grad_systems_per_wave", ctypes.c_int),
                ("grad_lds", ctypes.c_int)]


class _Model(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("parent", ctypes.c_void_p), ("jtype", ctypes.c_void_p),
                ("ncontacts", ctypes.c_int), ("contact_link", ctypes.c_void_p), ("mu", ctypes.c_double),
                ("beta", ctypes.c_double), ("niter", ctypes.c_int), ("gravity", ctypes.c_double * 3),
                ("limits", ctypes.c_void_p), ("tiling", ctypes.c_void_p)]


def pack_params(system, centers, radii) -> np.ndarray:
    """One system's parameter vector in the library's order: per link E_T
    (9), r_T (3), axis (3), mass, com (3), inertia about the com (6); then
    per sphere its centre (3) and radius."""
    rows = [np.concatenate([np.asarray(system.E_T[i], np.float64).reshape(9), system.r_T[i], system.axis[i],
                            [system.mass[i]], system.com[i], system.Ic[i]]) for i in range(system.n)]
    rows += [np.concatenate([np.asarray(c, np.float64).reshape(3), [r]]) for c, r in zip(centers, radii)]
    return np.concatenate(rows) if rows else np.zeros(0)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class ContactBatch:
    """B systems of one topology with contact spheres on links `contact_link`
    (per system: centers [B][nc][3] in link coordinates, radii [B][nc]);
    box friction mu, Baumgarte factor beta, niter PGS sweeps per solve."""

    def __init__(self, systems, contact_link, centers, radii, mu=0.5, beta=0.0, niter=30,
                 gravity=(0.0, -9.81, 0.0), dtype=torch.float32, device="cuda"):
        s0 = systems[0]
        for s in systems:
            if not (np.array_equal(s.parent, s0.parent) and np.array_equal(s.jtype, s0.jtype)):
                raise ValueError("ContactBatch: every system must share the first one's topology")
        # joint limits (lo, hi, k, d per link) are a model constant shared by the batch
        lim0 = getattr(s0, "limits", None)
        for s in systems:
            lim = getattr(s, "limits", None)
            if (lim is None) != (lim0 is None) or (lim is not None and not np.array_equal(lim, lim0)):
                raise ValueError("ContactBatch: every system must share the first one's joint limits")
        self.limits = None if lim0 is None else np.ascontiguousarray(np.asarray(lim0, np.float64).reshape(-1))
        self.parent = np.ascontiguousarray(s0.parent, dtype=np.int32)
        self.jtype = np.ascontiguousarray(s0.jtype, dtype=np.int32)
        self.clink = np.ascontiguousarray(np.asarray(contact_link, dtype=np.int32).reshape(-1))
        # launch geometry (sim_contact_tiling_t), kept alive with the model that points at it
        self._tiling = _Tiling(8, 16, 1)
        self.m = _Model(int(s0.n), self.parent.ctypes.data, self.jtype.ctypes.data, int(self.clink.size),
                        self.clink.ctypes.data if self.clink.size else None, float(mu), float(beta), int(niter),
                        (ctypes.c_double * 3)(*[float(g) for g in gravity]),
                        self.limits.ctypes.data if self.limits is not None else None, ctypes.addressof(self._tiling))
        nq, nv, nu, npar = (ctypes.c_int() for _ in range(4))
        N.check(N.lib().sim_contact_param_count(ctypes.byref(self.m), ctypes.byref(nq), ctypes.byref(nv),
                                                ctypes.byref(nu), ctypes.byref(npar)))
        self.nq, self.nv, self.nu, self.np = nq.value, nv.value, nu.value, npar.value
        P = np.stack([pack_params(s, c, r) for s, c, r in zip(systems, centers, radii)], axis=1)
        assert P.shape == (self.np, len(systems))
        self.B = len(systems)
        self.dtype = dtype
        self.P = torch.tensor(P, dtype=dtype, device=device)

    @property
    def tiling(self) -> dict:
        """Systems per wavefront of the rollout and of the gradient kernels,
        and whether the gradient keeps its working copies in LDS."""
        return {"rollout_systems_per_wave": self._tiling.rollout_systems_per_wave,
                "grad_systems_per_wave": self._tiling.grad_systems_per_wave, "grad_lds": self._tiling.grad_lds}

    def set_tiling(self, rollout_systems_per_wave: int = 8, grad_systems_per_wave: int = 16,
                   grad_lds: int = 1) -> None:
        """Launch geometry of the next calls (rollout: 8, 4 or 2; gradient: 16,
        8 or 4 with grad_lds 1, or 16 with grad_lds 0; the library rejects
        other values at the call)."""
        self._tiling.rollout_systems_per_wave = int(rollout_systems_per_wave)
        self._tiling.grad_systems_per_wave = int(grad_systems_per_wave)
        self._tiling.grad_lds = int(grad_lds)

    def autotune(self, q0, qd0, tau, dt) -> dict:
        """Times T = tau.shape[0] probe steps of the rollout and its gradient at
        every launch geometry (sim_contact_autotune), keeps the fastest and
        returns it with the ms per probe step of each kernel."""
        T = int(tau.shape[0])
        self._check(q0, (self.nq, self.B), "q0")
        self._check(qd0, (self.nv, self.B), "qd0")
        self._check(tau, (T, self.nu, self.B), "tau")
        chosen, rms, gms = _Tiling(), ctypes.c_double(), ctypes.c_double()
        N.check(N.lib().sim_contact_autotune(ctypes.byref(self.m), _DT[self.dtype], self.B, _ptr(self.P), _ptr(q0),
                                             _ptr(qd0), _ptr(tau), float(dt), T,
                                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                             ctypes.byref(chosen), ctypes.byref(rms), ctypes.byref(gms)))
        self.set_tiling(chosen.rollout_systems_per_wave, chosen.grad_systems_per_wave, chosen.grad_lds)
        return dict(self.tiling, rollout_ms_per_probe_step=rms.value, grad_ms_per_probe_step=gms.value)

    def _check(self, t, shape, name):
        if t.dtype != self.dtype or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: need a contiguous {self.dtype} CUDA tensor of shape {tuple(shape)}")

    def rollout(self, q0, qd0, tau, dt, traj=True, counts=False):
        """T = tau.shape[0] steps; returns qT, qdT and, as asked, the states
        x_0 .. x_T [T + 1][nq + nv][B] and the per-step contact counts [T][B]."""
        T = int(tau.shape[0])
        self._check(q0, (self.nq, self.B), "q0")
        self._check(qd0, (self.nv, self.B), "qd0")
        self._check(tau, (T, self.nu, self.B), "tau")
        qT, qdT = torch.empty_like(q0), torch.empty_like(qd0)
        tr = torch.empty((T + 1, self.nq + self.nv, self.B), dtype=self.dtype, device=q0.device) if traj else None
        nc = torch.empty((T, self.B), dtype=torch.int32, device=q0.device) if counts else None
        N.check(N.lib().sim_contact_rollout(ctypes.byref(self.m), _DT[self.dtype], self.B, _ptr(self.P), _ptr(q0),
                                            _ptr(qd0), _ptr(tau), float(dt), T, _ptr(tr), _ptr(qT), _ptr(qdT),
                                            _ptr(nc), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        out = (qT, qdT)
        if traj:
            out += (tr,)
        if counts:
            out += (nc,)
        return out

    def grad(self, traj, tau, dt, gqT, gqdT, mu_grad=False):
        """Gradient of <gqT, qT> + <gqdT, qdT> through the rollout that wrote
        traj: returns gq0 [nq][B], gqd0 [nv][B], gtau [T][nu][B] and, with
        mu_grad, dL/dmu per system [B]."""
        T = int(tau.shape[0])
        self._check(traj, (T + 1, self.nq + self.nv, self.B), "traj")
        self._check(tau, (T, self.nu, self.B), "tau")
        self._check(gqT, (self.nq, self.B), "gqT")
        self._check(gqdT, (self.nv, self.B), "gqdT")
        gq0, gqd0, gtau = torch.empty_like(gqT), torch.empty_like(gqdT), torch.empty_like(tau)
        gmu = torch.empty(self.B, dtype=self.dtype, device=gqT.device) if mu_grad else None
        N.check(N.lib().sim_contact_rollout_grad(ctypes.byref(self.m), _DT[self.dtype], self.B, _ptr(self.P),
                                                 _ptr(traj), _ptr(tau), float(dt), T, _ptr(gqT), _ptr(gqdT),
                                                 _ptr(gq0), _ptr(gqd0), _ptr(gtau), _ptr(gmu),
                                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        return (gq0, gqd0, gtau, gmu) if mu_grad else (gq0, gqd0, gtau)
