"""abadj: batched differentiable articulated-body dynamics for AMD MI355X.

Forward dynamics by the Articulated Body Algorithm, semi-implicit Euler time
stepping, and the checkpointed reverse-time adjoint, all in HIP kernels for
gfx950 behind the C ABI of include/abadj.h.  ``Sim`` and ``rollout`` load
the native library on first use; ``synth`` (seeded workload generators)
needs no GPU.
"""

__all__ = ["Sim", "rollout", "synth"]


def __getattr__(name):
    if name in ("Sim", "rollout"):
        from . import sim as _sim
        return getattr(_sim, name)
    raise AttributeError(name)
